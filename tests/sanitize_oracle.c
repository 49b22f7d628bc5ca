/* Driver for a sanitizer build of the CPU oracle (AddressSanitizer and UndefinedBehaviorSanitizer,
 * built with gcc by tests/test_sanitizers.py): random CSR inputs with empty rows and zero columns,
 * the product in every mode (values, pattern only, long double, split over threads, selected
 * rows), the adjoint on the product's pattern, every output released.  Prints "ok" at the end;
 * a sanitizer report or a nonzero return code fails the test. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_rap_ex(int32_t n, int32_t m1, int32_t m2, const int32_t* A_rowptr, const int32_t* A_col,
                  const double* A_val, const int32_t* Q1_rowptr, const int32_t* Q1_col,
                  const double* Q1_val, const int32_t* Q2_rowptr, const int32_t* Q2_col,
                  const double* Q2_val, const int32_t* rows, int32_t n_sel, int flags,
                  int32_t nthreads, int32_t** out_rowptr, int32_t** out_col, double** out_val,
                  double** out_abs, int64_t* out_nnz);
int oracle_ptap_backward(int32_t n, int32_t m, const int32_t* A_rowptr, const int32_t* A_col,
                         const double* A_val, const int32_t* P_rowptr, const int32_t* P_col,
                         const double* P_val, const int32_t* C_rowptr, const int32_t* C_col,
                         const double* W, double* dA, double* dP);
void oracle_free(void* p);

static uint64_t st = 0x9E3779B97F4A7C15ULL;
static uint32_t rnd(void) {  /* xorshift64* */
  st ^= st >> 12;
  st ^= st << 25;
  st ^= st >> 27;
  return (uint32_t)((st * 0x2545F4914F6CDD1DULL) >> 32);
}

/* Random CSR: rows x cols, each entry kept with probability pct/100, a tenth of the rows empty,
 * columns ascending. */
static void make(int rows, int cols, int pct, int32_t** rp, int32_t** c, double** v) {
  *rp = malloc(sizeof(int32_t) * (size_t)(rows + 1));
  *c = malloc(sizeof(int32_t) * (size_t)rows * (size_t)cols + 1);
  *v = malloc(sizeof(double) * (size_t)rows * (size_t)cols + 1);
  int k = 0;
  (*rp)[0] = 0;
  for (int r = 0; r < rows; ++r) {
    if (rnd() % 10 != 0)
      for (int j = 0; j < cols; ++j)
        if ((int)(rnd() % 100) < pct) {
          (*c)[k] = j;
          (*v)[k] = (double)((int)(rnd() % 2001) - 1000) / 1000.0;
          ++k;
        }
    (*rp)[r + 1] = k;
  }
}

int main(void) {
  for (int trial = 0; trial < 12; ++trial) {
    const int n = 5 + (int)(rnd() % 120), m = 1 + (int)(rnd() % 30);
    int32_t *Arp, *Ac, *Prp, *Pc;
    double *Av, *Pv;
    make(n, n, 4, &Arp, &Ac, &Av);
    make(n, m, 10, &Prp, &Pc, &Pv);
    int32_t sel[3] = {0, m - 1, m / 2};
    for (int mode = 0; mode < 5; ++mode) {
      int flags = mode == 1 ? 1 : mode == 2 ? 2 : 0;
      int threads = mode == 3 ? 7 : 1;
      const int32_t* rows = mode == 4 ? sel : NULL;
      int32_t *orp = NULL, *oc = NULL;
      double *ov = NULL, *oa = NULL;
      int64_t nnz = 0;
      int rc = oracle_rap_ex(n, m, m, Arp, Ac, Av, Prp, Pc, Pv, Prp, Pc, Pv, rows, rows ? 3 : 0, flags,
                             threads, &orp, &oc, &ov, &oa, &nnz);
      if (rc) {
        printf("oracle_rap_ex failed %d\n", rc);
        return 1;
      }
      if (mode == 0) {
        double* W = malloc(sizeof(double) * (size_t)(nnz + 1));
        double* dA = malloc(sizeof(double) * (size_t)(Arp[n] + 1));
        double* dP = malloc(sizeof(double) * (size_t)(Prp[n] + 1));
        for (int64_t q = 0; q < nnz; ++q) W[q] = (double)(q % 7) - 3.0;
        rc = oracle_ptap_backward(n, m, Arp, Ac, Av, Prp, Pc, Pv, orp, oc, W, dA, dP);
        free(W);
        free(dA);
        free(dP);
        if (rc) {
          printf("oracle_ptap_backward failed %d\n", rc);
          return 1;
        }
      }
      oracle_free(orp);
      oracle_free(oc);
      oracle_free(ov);
      oracle_free(oa);
    }
    free(Arp); free(Ac); free(Av); free(Prp); free(Pc); free(Pv);
  }
  printf("ok\n");
  return 0;
}
