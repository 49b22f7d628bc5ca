// Short-row adjoint kernel (dL/dA and dL/dP of C = P^T A P with dL/dC = dC), for fine rows I
// whose rows of dC under P(I,:) hold few entries in total.
//
// Per fine row I, one wavefront and one LDS table keyed by coarse column j, holding two values:
//   U_I(j) = sum_{i in P(I,:)} P(I,i) dC(i,j)    and    R_I(j) = (A P)(I,j).
// Every column of R_I is a column of U_I (C's pattern is the structural product, so R_I(j) != 0
// structurally implies C(i,j) for every i in P(I,:)), which lets both live under one key.
//   1. walk the entries of dC(i,:) for all i in P(I,:) as one flat range (up to four passes of
//      64 lanes): insert j, add P(I,i) dC(i,j) into U.  Each lane keeps (slot, dC value,
//      segment i) of the entries it walked.
//   2. walk the products (J, j) of row I of AP: with u = U_I(j),
//        dA(I,J) += u P(J,j)        (LDS accumulator per A entry, then one store),
//        dP(J,j) += A(I,J) u        (the A^T P dC term; device-wide atomic add),
//        R_I(j)  += A(I,J) P(J,j)   (the same slot: no second table and no second walk).
//   3. the A P dC^T term dP(I,i) += sum_j R_I(j) dC(i,j) from the entries kept in step 1: the
//      lanes of one segment i are summed by a segmented prefix sum over the wavefront.
// The general kernel (kernels.hip) forms R_I in a second table and reads dC's rows again; this
// one reads every input entry once per row.
#include "internal.hpp"

namespace ptapk {
namespace {

constexpr int kAdjWaves = 4;
constexpr int kAdjThreads = kAdjWaves * WAVE;

struct AdjScratch {
  int off[WAVE];       // product walk: first product number of each A entry of the chunk
  int ps[WAVE];        // start of row J of P for each A entry
  double a[WAVE];      // A(I,J)
  double dacc[WAVE];   // dA(I,J) being summed
  double dpacc[WAVE];  // A P dC^T term of dP(I, .) per entry of P(I,:)
};

// x taken from another lane by a DPP row operation; lanes without a source read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Inclusive sum of x over the lanes head..ln of this lane's segment (segments are runs of
// consecutive lanes, head = first lane of the run, head <= ln).  Shifts by 1, 2, 4, 8 within
// rows of 16 lanes, then the sums ending at lanes 15 and 47 are broadcast into rows 1 and 3, and
// the one ending at lane 31 into rows 2 and 3; a lane adds a shifted sum only if that sum's last
// lane lies in its own segment.  All 64 lanes must be active.
__device__ __forceinline__ double seg_incl_sum(double x, int ln, int head) {
  double t = dpp_f64<0x111, 0xF>(x);
  if (ln - 1 >= head) x += t;
  t = dpp_f64<0x112, 0xF>(x);
  if (ln - 2 >= head) x += t;
  t = dpp_f64<0x114, 0xF>(x);
  if (ln - 4 >= head) x += t;
  t = dpp_f64<0x118, 0xF>(x);
  if (ln - 8 >= head) x += t;
  t = dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  if ((ln & 16) && (ln & ~15) - 1 >= head) x += t;
  t = dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  if ((ln & 32) && 31 >= head) x += t;
  return x;
}

__global__ __launch_bounds__(kAdjThreads) void k_backward_short(NumericArgs a,
                                                                const double* __restrict__ dC,
                                                                double* dA, double* dP,
                                                                const int* __restrict__ rows,
                                                                int count, int cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int ln = lane();
  AdjScratch* ws = reinterpret_cast<AdjScratch*>(smem) + wid;
  unsigned char* tab = smem + kAdjWaves * sizeof(AdjScratch);
  double* U = reinterpret_cast<double*>(tab) + (size_t)wid * 2 * cap;
  double* R = U + cap;
  int* keys = reinterpret_cast<int*>(tab + (size_t)kAdjWaves * 2 * cap * sizeof(double)) + wid * cap;
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  const Patterns& p = a.p;
  for (int s = ln; s < cap; s += WAVE) {
    keys[s] = EMPTY;
    U[s] = 0.0;
    R[s] = 0.0;
  }
  wave_sync();

  for (int r = blockIdx.x * kAdjWaves + wid; r < count; r += gridDim.x * kAdjWaves) {
    const int I = rows[r];
    const int p0 = p.P_rowptr[I];
    const int np = p.P_rowptr[I + 1] - p0;  // 1 <= np <= 64 for the rows of this kernel
    const int a0 = p.A_rowptr[I], a1 = p.A_rowptr[I + 1];

    // 1. U_I over the flat range of dC's entries
    int cs = 0, cl = 0;
    double w = 0.0;
    if (ln < np) {
      const int i = p.P_col[p0 + ln];
      cs = a.C_rowptr[i];
      cl = a.C_rowptr[i + 1] - cs;
      w = a.P_val[p0 + ln];
      ws->dpacc[ln] = 0.0;
    }
    const int incl = wave_incl_scan(cl);
    const int excl = incl - cl;
    const int nw = __builtin_amdgcn_readlane(incl, WAVE - 1);  // <= kAdjMaxWalk
    int sl[kAdjPasses], sgv[kAdjPasses], hd[kAdjPasses];
    bool en[kAdjPasses];
    double xv[kAdjPasses];
#pragma unroll
    for (int ps = 0; ps < kAdjPasses; ++ps) {
      sl[ps] = -1;
      sgv[ps] = 0;
      hd[ps] = 0;
      en[ps] = false;
      xv[ps] = 0.0;
      if (ps * WAVE < nw) {
        const int q = ps * WAVE + ln;
        int sg = 0;
        for (int e = 1; e < np; ++e) sg += q >= __builtin_amdgcn_readlane(excl, e) ? 1 : 0;
        const int so = __shfl(excl, sg, WAVE), se = __shfl(incl, sg, WAVE);
        const int sc = __shfl(cs, sg, WAVE);
        const double sw = __shfl(w, sg, WAVE);
        hd[ps] = max(so - ps * WAVE, 0);
        en[ps] = q + 1 == se || ln == WAVE - 1;
        sgv[ps] = sg;
        if (q < nw) {
          const int c = sc + (q - so);
          const double x = dC[c];
          bool fresh;
          const int s = hs_insert<false>(keys, mask, shift, a.C_col[c], fresh);
          atomicAdd(U + s, sw * x);
          sl[ps] = s;
          xv[ps] = x;
        }
      }
    }
    wave_sync();

    // 2. products (J, j): dA(I,J), the A^T P dC term of dP, and R_I
    for (int base = a0; base < a1; base += WAVE) {
      const int t = base + ln;
      int ps = 0, pl = 0;
      double av = 0.0;
      if (t < a1) {
        const int J = p.A_col[t];
        ps = p.P_rowptr[J];
        pl = p.P_rowptr[J + 1] - ps;
        av = a.A_val[t];
      }
      const int pincl = wave_incl_scan(pl);
      const int total = __builtin_amdgcn_readlane(pincl, WAVE - 1);
      ws->off[ln] = pincl - pl;
      ws->ps[ln] = ps;
      ws->a[ln] = av;
      ws->dacc[ln] = 0.0;
      wave_sync();
      for (int q = ln; q < total; q += WAVE) {
        int lo = 0;
#pragma unroll
        for (int step = WAVE / 2; step > 0; step >>= 1)
          if (ws->off[lo + step] <= q) lo += step;
        const int k = ws->ps[lo] + (q - ws->off[lo]);
        const double pv = a.P_val[k];
        const int s = hs_find<false>(keys, mask, shift, p.P_col[k]);
        if (s >= 0) {
          const double u = U[s];
          const double aj = ws->a[lo];
          if (dA) atomicAdd(ws->dacc + lo, u * pv);
          if (dP) {
            unsafeAtomicAdd(dP + k, aj * u);
            atomicAdd(R + s, aj * pv);
          }
        }
      }
      wave_sync();
      if (dA && t < a1) dA[t] = ws->dacc[ln];
      wave_sync();
    }

    // 3. the A P dC^T term: dP(I,i) += sum over the walked entries of segment i of R_I(j) dC(i,j)
    if (dP) {
#pragma unroll
      for (int ps = 0; ps < kAdjPasses; ++ps) {
        if (ps * WAVE < nw) {
          double y = sl[ps] >= 0 ? R[sl[ps]] * xv[ps] : 0.0;
          y = seg_incl_sum(y, ln, hd[ps]);
          if (sl[ps] >= 0 && en[ps]) atomicAdd(ws->dpacc + sgv[ps], y);
        }
      }
      wave_sync();
      if (ln < np) unsafeAtomicAdd(dP + p0 + ln, ws->dpacc[ln]);
    }

    // clear the slots this row used
#pragma unroll
    for (int ps = 0; ps < kAdjPasses; ++ps)
      if (sl[ps] >= 0) {
        keys[sl[ps]] = EMPTY;
        U[sl[ps]] = 0.0;
        R[sl[ps]] = 0.0;
      }
    wave_sync();
  }
}

}  // namespace

size_t backward_short_lds_bytes(int cap) {
  return (size_t)kAdjWaves * (sizeof(AdjScratch) + (size_t)cap * (2 * sizeof(double) + sizeof(int)));
}

hipError_t launch_backward_short(const NumericArgs& a, const double* dC, double* dA, double* dP,
                                 const RowClass& rc, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  if (rc.global || rc.cap > kAdjMaxCap) return hipErrorInvalidValue;
  const long long g = ((long long)rc.count + kAdjWaves - 1) / kAdjWaves;
  const int grid = (int)std::min<long long>(g, 1 << 30);
  hipLaunchKernelGGL(k_backward_short, dim3(grid), dim3(kAdjThreads), backward_short_lds_bytes(rc.cap),
                     s, a, dC, dA, dP, rc.rows, rc.count, rc.cap);
  return hipGetLastError();
}

}  // namespace ptapk
