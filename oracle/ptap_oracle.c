/*
 * CPU oracle for the sparse triple product C = P^T A P and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct reference the
 * GPU library is checked against.  It shares no code, header, table or helper with the
 * GPU library, and only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it.
 *
 * Arithmetic: IEEE binary64 (a long double diagnostic mode exists for the product), no
 * blocking, no reordering beyond what the definitions below state.  The product can split its
 * output rows over threads; each row is computed the same way whichever thread runs it.
 *
 * Matrices are CSR with int32 row pointers and column indices (sorted, unique within a
 * row) and double values.  Every function returns 0 on success and a negative number on
 * an allocation failure or malformed input.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n_rows, n_cols;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val; /* may be NULL when only the pattern is needed */
} ocsr;

/* Column lists of a CSR matrix (its pattern transpose), built by a counting sort.
 * For column c the rows r with M(r,c) stored are t_row[t_ptr[c] .. t_ptr[c+1]) in
 * ascending order, and t_src[k] is the position of that entry in M's CSR arrays. */
typedef struct {
  int32_t* t_ptr;
  int32_t* t_row;
  int64_t* t_src;
} ocols;

static void free_cols(ocols* t) {
  free(t->t_ptr);
  free(t->t_row);
  free(t->t_src);
}

static int build_cols(const ocsr* M, ocols* t) {
  int64_t nnz = M->rowptr[M->n_rows];
  t->t_ptr = (int32_t*)calloc((size_t)M->n_cols + 1, sizeof(int32_t));
  t->t_row = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  t->t_src = (int64_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
  int32_t* cursor = (int32_t*)malloc(((size_t)M->n_cols + 1) * sizeof(int32_t));
  if (!t->t_ptr || !t->t_row || !t->t_src || !cursor) {
    free(cursor);
    free_cols(t);
    return -1;
  }
  for (int64_t k = 0; k < nnz; ++k) t->t_ptr[M->col[k] + 1]++;
  for (int32_t c = 0; c < M->n_cols; ++c) t->t_ptr[c + 1] += t->t_ptr[c];
  memcpy(cursor, t->t_ptr, ((size_t)M->n_cols + 1) * sizeof(int32_t));
  /* Rows are visited in ascending order, so every column list comes out ascending. */
  for (int32_t r = 0; r < M->n_rows; ++r) {
    for (int32_t k = M->rowptr[r]; k < M->rowptr[r + 1]; ++k) {
      int32_t c = M->col[k];
      t->t_row[cursor[c]] = r;
      t->t_src[cursor[c]] = k;
      cursor[c]++;
    }
  }
  free(cursor);
  return 0;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Growable output row storage. */
typedef struct {
  int32_t* col;
  double* val;
  double* absv;
  int64_t len, cap;
} obuf;

static int obuf_push(obuf* b, int32_t c, double v, double a) {
  if (b->len == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 1024;
    int32_t* c2 = (int32_t*)realloc(b->col, (size_t)nc * sizeof(int32_t));
    if (!c2) return -1;
    b->col = c2;
    double* v2 = (double*)realloc(b->val, (size_t)nc * sizeof(double));
    if (!v2) return -1;
    b->val = v2;
    double* a2 = (double*)realloc(b->absv, (size_t)nc * sizeof(double));
    if (!a2) return -1;
    b->absv = a2;
    b->cap = nc;
  }
  b->col[b->len] = c;
  b->val[b->len] = v;
  b->absv[b->len] = a;
  b->len++;
  return 0;
}

void oracle_free(void* p) { free(p); }

/*
 * General Galerkin-type product C = Q1^T A Q2 (A is n x n, Q1 is n x m1, Q2 is n x m2),
 * evaluated in the row form of the all-at-once formula (Section 3, Eq. allatonce and
 * Eq. allatoncerow): for each output row i,
 *
 *     C(i, :) = sum over I with Q1(I,i) stored of  Q1(I,i) * ( sum over J in row I of A
 *               of A(I,J) * Q2(J, :) ).
 *
 * The pattern is the structural product: (i, j) is stored whenever some I, J have
 * Q1(I,i), A(I,J) and Q2(J,j) all stored, whatever the values (explicit zeros count and
 * exact cancellation drops nothing), because the symbolic phase uses no floating point
 * (Section 2, the symbolic/numeric split).  Columns come out ascending within each row.
 *
 * Besides C the oracle returns, on the same pattern, Cabs = |Q1|^T |A| |Q2|, the sum of the
 * magnitudes of every product term, which bounds the rounding error of any summation order.
 *
 * Every output row is computed on its own (the terms of row i, in the order above, into one
 * accumulator per column), so splitting the rows over threads cannot change a single bit.
 */

/* Inputs and options shared by the row workers. */
typedef struct {
  int32_t m1, m2;
  const int32_t *A_rowptr, *A_col;
  const double* A_val;
  const double* Q1_val;
  const int32_t *Q2_rowptr, *Q2_col;
  const double* Q2_val;
  const ocols* q1c;
  const int32_t* rows; /* NULL: output row r is row r of C */
  int pattern_only;
  int long_double;     /* accumulate in long double, round once at the end */
} rap_job;

/* Rows [r0, r1) of the output into out (columns, values, bounds) and len[r - r0] = the
 * number of entries of row r.  Returns 0, -1 on allocation failure, -2 on a bad row index. */
typedef struct {
  const rap_job* job;
  int32_t r0, r1;
  int64_t* len;
  obuf out;
  int rc;
} rap_part;

static int rap_rows(rap_part* part) {
  const rap_job* jb = part->job;
  const ocols* q1c = jb->q1c;
  const int pattern_only = jb->pattern_only;
  const int32_t* A_rowptr = jb->A_rowptr;
  const int32_t* A_col = jb->A_col;
  const double* A_val = jb->A_val;
  const double* Q1_val = jb->Q1_val;
  const int32_t* Q2_rowptr = jb->Q2_rowptr;
  const int32_t* Q2_col = jb->Q2_col;
  const double* Q2_val = jb->Q2_val;
  const size_t m2 = (size_t)jb->m2;
  double* acc = (double*)calloc(m2 + 1, sizeof(double));
  long double* accl = jb->long_double ? (long double*)calloc(m2 + 1, sizeof(long double)) : NULL;
  double* absacc = (double*)calloc(m2 + 1, sizeof(double));
  char* mark = (char*)calloc(m2 + 1, 1);
  int32_t* touched = (int32_t*)malloc((m2 + 1) * sizeof(int32_t));
  int rc = 0;
  if (!acc || !absacc || !mark || !touched || (jb->long_double && !accl)) {
    rc = -1;
    goto done;
  }
  for (int32_t r = part->r0; r < part->r1; ++r) {
    int32_t i = jb->rows ? jb->rows[r] : r;
    if (i < 0 || i >= jb->m1) {
      rc = -2;
      goto done;
    }
    int32_t ntouched = 0;
    for (int32_t t = q1c->t_ptr[i]; t < q1c->t_ptr[i + 1]; ++t) {
      int32_t I = q1c->t_row[t];
      double w = pattern_only ? 0.0 : Q1_val[q1c->t_src[t]];
      for (int32_t ka = A_rowptr[I]; ka < A_rowptr[I + 1]; ++ka) {
        int32_t J = A_col[ka];
        double a = pattern_only ? 0.0 : A_val[ka];
        for (int32_t kp = Q2_rowptr[J]; kp < Q2_rowptr[J + 1]; ++kp) {
          int32_t j = Q2_col[kp];
          if (!mark[j]) {
            mark[j] = 1;
            touched[ntouched++] = j;
          }
          if (pattern_only) continue;
          double p = Q2_val[kp];
          if (accl)
            accl[j] += (long double)w * ((long double)a * (long double)p);
          else
            acc[j] += w * (a * p);
          absacc[j] += fabs(w) * (fabs(a) * fabs(p));
        }
      }
    }
    qsort(touched, (size_t)ntouched, sizeof(int32_t), cmp_i32);
    for (int32_t t = 0; t < ntouched; ++t) {
      int32_t j = touched[t];
      double v = accl ? (double)accl[j] : acc[j];
      if (obuf_push(&part->out, j, v, absacc[j])) {
        rc = -1;
        goto done;
      }
      acc[j] = 0.0;
      if (accl) accl[j] = 0.0L;
      absacc[j] = 0.0;
      mark[j] = 0;
    }
    part->len[r - part->r0] = ntouched;
  }
done:
  free(acc);
  free(accl);
  free(absacc);
  free(mark);
  free(touched);
  part->rc = rc;
  return rc;
}

static void* rap_thread(void* arg) {
  rap_rows((rap_part*)arg);
  return NULL;
}

/*
 * rows / n_sel: if rows is NULL every output row 0..m1-1 is produced; otherwise only the
 * listed rows, in the listed order (out_rowptr then has n_sel+1 entries).
 * flags: ORACLE_PATTERN_ONLY skips the values (out_val and out_abs are returned as NULL);
 * ORACLE_LONG_DOUBLE sums every row's terms in long double (x86 80-bit extended, 64-bit
 * significand) and rounds each entry to double once, a diagnostic of the FP64 sums' own error.
 * nthreads: the output rows are cut into that many contiguous ranges, one POSIX thread each;
 * the result is identical bit for bit to nthreads = 1.
 *
 * Output arrays are allocated here with malloc and released with oracle_free.
 */
#define ORACLE_PATTERN_ONLY 1
#define ORACLE_LONG_DOUBLE 2

int oracle_rap_ex(int32_t n, int32_t m1, int32_t m2, const int32_t* A_rowptr, const int32_t* A_col,
                  const double* A_val, const int32_t* Q1_rowptr, const int32_t* Q1_col,
                  const double* Q1_val, const int32_t* Q2_rowptr, const int32_t* Q2_col,
                  const double* Q2_val, const int32_t* rows, int32_t n_sel, int flags,
                  int32_t nthreads, int32_t** out_rowptr, int32_t** out_col, double** out_val,
                  double** out_abs, int64_t* out_nnz) {
  const int pattern_only = (flags & ORACLE_PATTERN_ONLY) != 0;
  ocsr Q1 = {n, m1, Q1_rowptr, Q1_col, Q1_val};
  ocols q1c;
  if (build_cols(&Q1, &q1c)) return -1;
  int32_t nrows_out = rows ? n_sel : m1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > nrows_out) nthreads = nrows_out > 0 ? nrows_out : 1;
  rap_job job = {m1, m2, A_rowptr, A_col, A_val, Q1_val, Q2_rowptr, Q2_col, Q2_val, &q1c, rows,
                 pattern_only, (flags & ORACLE_LONG_DOUBLE) != 0 && !pattern_only};
  int32_t* rp = (int32_t*)malloc(((size_t)nrows_out + 1) * sizeof(int32_t));
  int64_t* len = (int64_t*)calloc((size_t)nrows_out + 1, sizeof(int64_t));
  rap_part* parts = (rap_part*)calloc((size_t)nthreads, sizeof(rap_part));
  pthread_t* tid = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  char* started = (char*)calloc((size_t)nthreads, 1);
  obuf out = {0};
  int rc = 0;
  if (!rp || !len || !parts || !tid || !started) {
    rc = -1;
    goto done;
  }
  for (int32_t k = 0; k < nthreads; ++k) {
    parts[k].job = &job;
    parts[k].r0 = (int32_t)(((int64_t)nrows_out * k) / nthreads);
    parts[k].r1 = (int32_t)(((int64_t)nrows_out * (k + 1)) / nthreads);
    parts[k].len = len + parts[k].r0;
  }
  if (nthreads == 1) {
    rap_rows(&parts[0]);
  } else {
    for (int32_t k = 0; k < nthreads; ++k)
      started[k] = pthread_create(&tid[k], NULL, rap_thread, &parts[k]) == 0;
    for (int32_t k = 0; k < nthreads; ++k) {
      if (started[k])
        pthread_join(tid[k], NULL);
      else
        rap_rows(&parts[k]); /* no thread could be started: run the range here */
    }
  }
  /* concatenate the parts in row order */
  int64_t total = 0;
  for (int32_t k = 0; k < nthreads; ++k) {
    if (parts[k].rc) {
      rc = parts[k].rc;
      goto done;
    }
    total += parts[k].out.len;
  }
  if (total > INT32_MAX) {
    rc = -3;
    goto done;
  }
  rp[0] = 0;
  for (int32_t r = 0; r < nrows_out; ++r) rp[r + 1] = rp[r] + (int32_t)len[r];
  if (nthreads == 1) {
    out = parts[0].out;
    parts[0].out = (obuf){0};
  } else {
    out.cap = total > 0 ? total : 1;
    out.col = (int32_t*)malloc((size_t)out.cap * sizeof(int32_t));
    out.val = (double*)malloc((size_t)out.cap * sizeof(double));
    out.absv = (double*)malloc((size_t)out.cap * sizeof(double));
    if (!out.col || !out.val || !out.absv) {
      rc = -1;
      goto done;
    }
    for (int32_t k = 0; k < nthreads; ++k) {
      const obuf* b = &parts[k].out;
      if (!b->len) continue;
      memcpy(out.col + out.len, b->col, (size_t)b->len * sizeof(int32_t));
      memcpy(out.val + out.len, b->val, (size_t)b->len * sizeof(double));
      memcpy(out.absv + out.len, b->absv, (size_t)b->len * sizeof(double));
      out.len += b->len;
    }
  }
done:
  free_cols(&q1c);
  free(len);
  free(tid);
  free(started);
  if (parts) {
    for (int32_t k = 0; k < nthreads; ++k) {
      free(parts[k].out.col);
      free(parts[k].out.val);
      free(parts[k].out.absv);
    }
    free(parts);
  }
  if (rc) {
    free(rp);
    free(out.col);
    free(out.val);
    free(out.absv);
    return rc;
  }
  if (!out.col) { /* empty result: still hand back valid pointers */
    out.col = (int32_t*)malloc(sizeof(int32_t));
    out.val = (double*)malloc(sizeof(double));
    out.absv = (double*)malloc(sizeof(double));
  }
  *out_rowptr = rp;
  *out_col = out.col;
  *out_nnz = out.len;
  if (pattern_only) {
    free(out.val);
    free(out.absv);
    *out_val = NULL;
    *out_abs = NULL;
  } else {
    *out_val = out.val;
    *out_abs = out.absv;
  }
  return 0;
}

/* The product above in FP64 on one thread (pattern_only: skip the values). */
int oracle_rap(int32_t n, int32_t m1, int32_t m2, const int32_t* A_rowptr, const int32_t* A_col,
               const double* A_val, const int32_t* Q1_rowptr, const int32_t* Q1_col,
               const double* Q1_val, const int32_t* Q2_rowptr, const int32_t* Q2_col,
               const double* Q2_val, const int32_t* rows, int32_t n_sel, int pattern_only,
               int32_t** out_rowptr, int32_t** out_col, double** out_val, double** out_abs,
               int64_t* out_nnz) {
  return oracle_rap_ex(n, m1, m2, A_rowptr, A_col, A_val, Q1_rowptr, Q1_col, Q1_val, Q2_rowptr,
                       Q2_col, Q2_val, rows, n_sel, pattern_only ? ORACLE_PATTERN_ONLY : 0, 1,
                       out_rowptr, out_col, out_val, out_abs, out_nnz);
}

/* Value of W(i, j) on the pattern of C, zero off it (binary search in row i). */
static double w_at(const int32_t* C_rowptr, const int32_t* C_col, const double* W, int32_t i,
                   int32_t j) {
  int32_t lo = C_rowptr[i], hi = C_rowptr[i + 1];
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (C_col[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < C_rowptr[i + 1] && C_col[lo] == j) ? W[lo] : 0.0;
}

/*
 * Adjoint of C = P^T A P (Section 3, Eq. tripleproduct) for the loss L = sum over the
 * stored entries of C of W(i,j) * C(i,j), i.e. dL/dC = W on the pattern of C.
 *
 * Writing C(i,j) = sum_{I,J} P(I,i) A(I,J) P(J,j) and differentiating term by term:
 *
 *   dL/dA(I,J) = sum_{i in row I of P} sum_{j in row J of P} P(I,i) W(i,j) P(J,j)
 *                (the entries of P W P^T), evaluated on the pattern of A only;
 *
 *   dL/dP(K,k) = sum_{J in row K of A} A(K,J) sum_{j in row J of P} W(k,j) P(J,j)
 *                  (the I = K, i = k terms: entries of A P W^T)
 *              + sum_{I with A(I,K) stored} A(I,K) sum_{i in row I of P} P(I,i) W(i,k)
 *                  (the J = K, j = k terms: entries of A^T P W),
 *                evaluated on the pattern of P only.
 *
 * dA has A's nnz entries in A's CSR order, dP has P's nnz entries in P's CSR order; both are
 * caller-allocated and overwritten.
 */
int oracle_ptap_backward(int32_t n, int32_t m, const int32_t* A_rowptr, const int32_t* A_col,
                         const double* A_val, const int32_t* P_rowptr, const int32_t* P_col,
                         const double* P_val, const int32_t* C_rowptr, const int32_t* C_col,
                         const double* W, double* dA, double* dP) {
  (void)m;
  /* dA */
  for (int32_t I = 0; I < n; ++I) {
    for (int32_t ka = A_rowptr[I]; ka < A_rowptr[I + 1]; ++ka) {
      int32_t J = A_col[ka];
      double s = 0.0;
      for (int32_t ki = P_rowptr[I]; ki < P_rowptr[I + 1]; ++ki) {
        int32_t i = P_col[ki];
        for (int32_t kj = P_rowptr[J]; kj < P_rowptr[J + 1]; ++kj) {
          int32_t j = P_col[kj];
          s += P_val[ki] * w_at(C_rowptr, C_col, W, i, j) * P_val[kj];
        }
      }
      dA[ka] = s;
    }
  }
  /* dP, first term: rows of A P W^T */
  for (int32_t K = 0; K < n; ++K) {
    for (int32_t kk = P_rowptr[K]; kk < P_rowptr[K + 1]; ++kk) {
      int32_t k = P_col[kk];
      double s = 0.0;
      for (int32_t ka = A_rowptr[K]; ka < A_rowptr[K + 1]; ++ka) {
        int32_t J = A_col[ka];
        for (int32_t kj = P_rowptr[J]; kj < P_rowptr[J + 1]; ++kj)
          s += A_val[ka] * (w_at(C_rowptr, C_col, W, k, P_col[kj]) * P_val[kj]);
      }
      dP[kk] = s;
    }
  }
  /* dP, second term: rows of A^T P W, using A's column lists */
  ocsr Am = {n, n, A_rowptr, A_col, A_val};
  ocols at;
  if (build_cols(&Am, &at)) return -1;
  for (int32_t K = 0; K < n; ++K) {
    for (int32_t kk = P_rowptr[K]; kk < P_rowptr[K + 1]; ++kk) {
      int32_t k = P_col[kk];
      double s = 0.0;
      for (int32_t t = at.t_ptr[K]; t < at.t_ptr[K + 1]; ++t) {
        int32_t I = at.t_row[t];
        double a = A_val[at.t_src[t]];
        for (int32_t ki = P_rowptr[I]; ki < P_rowptr[I + 1]; ++ki)
          s += a * (P_val[ki] * w_at(C_rowptr, C_col, W, P_col[ki], k));
      }
      dP[kk] += s;
    }
  }
  free_cols(&at);
  return 0;
}
