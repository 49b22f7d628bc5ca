// Row-times-matrix products, short-row form.  In product mode, the two numeric products of the
// two-step method (Alg. 6), each row O(r,:) = sum_k X(r,k) Y(k,:) written into O's stored,
// sorted pattern:
//   AP = A P          X = A,    Y = P,   O = AP   (the stored auxiliary matrix, Alg. 4 rows)
//   C  = P^T (AP)     X = P^T,  Y = AP,  O = C    (rows of P^T: the column lists of P with the
//                                                  gathered values of its entries)
// In fold mode, the all-at-once product with the atomic fold: X = A, Y = P give R_I, and
// C(i,:) += P(I,i) R_I for every entry of P(I,:) (Eq. allatonceoutproduct) with device FP64
// atomics on C's pattern.
//
// Two rows per wavefront, one per 32-lane half, in the manner of the owner fold's short-row
// kernel: lane `sub` holds X(r, x0+sub) and the extent of row k of Y; the products X(r,k) Y(k,j)
// are dealt out 32 per step over the half (a prefix sum of the lengths of the rows of Y gives each
// lane its product and its segment), the gathers of four steps are issued together, and the
// products are added into the half's 64-slot LDS table (longer rows of X are taken 32 entries at
// a time by a second instantiation).  Then the half writes O's row (product mode) or folds (fold
// mode).  Rows with at most 32 keys; longer rows take the general kernels.  A wavefront works
// through a contiguous run of row pairs, whose row headers (row, extents in X and in O) lane
// h*32+k loads for iteration it0+k once per 32 iterations.
#include "internal.hpp"
#include "short_rows.hpp"

namespace ptapk {
namespace {

constexpr int kRmWaves = 8;
constexpr int kRmPrefetch = 4;  // product-walk steps whose loads are issued together
constexpr int kFoldBatch = 4;   // atomic fold: entries of P(I,:) whose columns are loaded together

struct RmHeader {
  int r, x0, x1, o0, o1;  // row of O (or -1), its extents in X and in O
};

__device__ __forceinline__ RmHeader rm_hdr_get(const RmHeader& b, int k, int half) {
  const int src = (half * kHalf + k) * 4;
  RmHeader h;
  h.r = __builtin_amdgcn_ds_bpermute(src, b.r);
  h.x0 = __builtin_amdgcn_ds_bpermute(src, b.x0);
  h.x1 = __builtin_amdgcn_ds_bpermute(src, b.x1);
  h.o0 = __builtin_amdgcn_ds_bpermute(src, b.o0);
  h.o1 = __builtin_amdgcn_ds_bpermute(src, b.o1);
  return h;
}

template <bool LONG, bool FOLD>
__global__ __launch_bounds__(kRmWaves * WAVE) void k_rowmul_short(RowMulArgs g,
                                                                  const int* __restrict__ rows,
                                                                  int count, int pairs_per_wave) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int half = ln / kHalf, sub = ln % kHalf;
  HalfScratch* hs = reinterpret_cast<HalfScratch*>(smem) + wid;
  int* keys = hs->keys[half];
  double* vals = hs->vals[half];
  keys[sub] = EMPTY;
  keys[sub + kHalf] = EMPTY;
  vals[sub] = 0.0;
  vals[sub + kHalf] = 0.0;

  const __amdgpu_buffer_rsrc_t rXp = buffer_rsrc(g.X_rowptr, (unsigned)(g.nX + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rXc = buffer_rsrc(g.X_col, (unsigned)g.nnzX * 4u);
  const __amdgpu_buffer_rsrc_t rXv = buffer_rsrc(g.X_val, (unsigned)g.nnzX * 8u);
  const __amdgpu_buffer_rsrc_t rYp = buffer_rsrc(g.Y_rowptr, (unsigned)(g.nY + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rYc = buffer_rsrc(g.Y_col, (unsigned)g.nnzY * 4u);
  const __amdgpu_buffer_rsrc_t rYv = buffer_rsrc(g.Y_val, (unsigned)g.nnzY * 8u);
  const __amdgpu_buffer_rsrc_t rOp = buffer_rsrc(g.O_rowptr, (unsigned)(g.nX + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rOc = buffer_rsrc(g.O_col, (unsigned)g.nnzO * 4u);
  const __amdgpu_buffer_rsrc_t rFv = buffer_rsrc(g.F_val, FOLD ? (unsigned)g.nnzO * 8u : 0u);
  const __amdgpu_buffer_rsrc_t rFp = buffer_rsrc(g.F_rowptr, FOLD ? (unsigned)(g.nF + 1) * 4u : 0u);
  const __amdgpu_buffer_rsrc_t rFc = buffer_rsrc(g.F_col, FOLD ? (unsigned)g.nnzF * 4u : 0u);
  wave_sync();

  const int npairs = (count + 1) / 2;
  const long long gw = (long long)blockIdx.x * kRmWaves + wid;
  const long long pb0 = gw * pairs_per_wave;
  const int pb = (int)(pb0 < npairs ? pb0 : npairs);
  const int pe = (int)(pb + (long long)pairs_per_wave < npairs ? pb + pairs_per_wave : npairs);
  RmHeader hb{-1, 0, 0, 0, 0};
  for (int pr = pb; pr < pe; ++pr) {
    const int k = (pr - pb) % kHalf;
    if (k == 0) {
      // headers of the next 32 pairs: lane h*32+k2 loads row 2*(pr+k2)+h
      const int ri = 2 * (pr + sub) + half;
      hb = RmHeader{-1, 0, 0, 0, 0};
      if (pr + sub < pe && ri < count) {
        hb.r = rows[ri];
        const v2u xp = ld_pair(rXp, hb.r), op = ld_pair(rOp, hb.r);
        hb.x0 = (int)xp[0];
        hb.x1 = (int)xp[1];
        hb.o0 = (int)op[0];
        hb.o1 = (int)op[1];
      }
    }
    const RmHeader h = rm_hdr_get(hb, k, half);

    // X(r,:) 32 entries at a time (one chunk unless LONG): lane sub holds X(r, xb+sub) and the
    // extent of its row of Y; the chunk's products, 32 per step and half, go into the table (the
    // first kRmPrefetch steps' gathers are issued together)
    const int xl = h.x1 - h.x0;
    auto chunk = [&](int xb) {
      const int t = xb + sub < xl ? h.x0 + xb + sub : -1;
      const int kc = ld_i32(rXc, t);
      const double w = ld_dbl(rXv, t);
      const v2u yp = ld_pair(rYp, t >= 0 ? kc : -1);
      const int len = (int)yp[1] - (int)yp[0];  // 0 where there is no entry (the load returned 0)
      const int incl = half_incl_scan(len);
      const int T0 = __builtin_amdgcn_readlane(incl, kHalf - 1), T1 = __builtin_amdgcn_readlane(incl, WAVE - 1);
      const int Th = half ? T1 : T0;
      const unsigned long long nonempty = ballot(len > 0);
      if (len > 0) {
        const int rk = prefix_count(nonempty) - (half ? __popc((unsigned)nonempty) : 0);
        hs->rec[half][rk] = SegRec{w, (int)yp[0] - (incl - len), 0};
      }
      wave_sync();
      const int nstep = (max(T0, T1) + kHalf - 1) / kHalf;
      int before = 0;
      ProdLoad pq[kRmPrefetch];
#pragma unroll
      for (int u = 0; u < kRmPrefetch; ++u)
        pq[u] = u < nstep ? prod_load(u, incl, len, Th, sub, half, before, hs->rec[half], rYc, rYv)
                          : ProdLoad{0, 0.0, 0.0, false};
#pragma unroll
      for (int u = 0; u < kRmPrefetch; ++u)
        if (pq[u].ok) hash_add64(keys, vals, pq[u].j, pq[u].w * pq[u].v);
      for (int st = kRmPrefetch; st < nstep; ++st) {
        const ProdLoad cu = prod_load(st, incl, len, Th, sub, half, before, hs->rec[half], rYc, rYv);
        if (cu.ok) hash_add64(keys, vals, cu.j, cu.w * cu.v);
      }
      wave_sync();
    };
    if constexpr (LONG) {
      // a loop around the walk costs the one-chunk rows about half their speed (measured), so
      // rows with at most 32 entries in X(r,:) use the other instantiation
      const int xlmax = max(__builtin_amdgcn_readlane(xl, 0), __builtin_amdgcn_readlane(xl, kHalf));
      for (int xb = 0; xb < xlmax; xb += kHalf) chunk(xb);
    } else {
      chunk(0);
    }

    if constexpr (FOLD) {
      // the atomic fold: C(i,:) += P(I,i) R_I for every entry P(I,i) (O's row r = P(I,:)); lane
      // sub holds entry sub's weight and the extent of row i of C, and each step takes kFoldBatch
      // entries of both halves: their column loads go out together, then every lane of a half
      // looks its column up in R_I and adds into C with a device-wide FP64 atomic
      const int npi = h.o1 - h.o0;
      const int e = sub < npi ? h.o0 + sub : -1;
      const int ci = ld_i32(rOc, e);
      const double cw = ld_dbl(rFv, e);
      const v2u cp = ld_pair(rFp, e >= 0 ? ci : -1);
      const int cc0 = (int)cp[0], cc1 = (int)cp[1];
      const long long cwb = __double_as_longlong(cw);
      const int cwl = (int)cwb, cwh = (int)(cwb >> 32);
      const int nmax = max(__builtin_amdgcn_readlane(npi, 0), __builtin_amdgcn_readlane(npi, kHalf));
      for (int kb = 0; kb < nmax; kb += kFoldBatch) {
        int cix[kFoldBatch], jj[kFoldBatch];
        double ww[kFoldBatch];
#pragma unroll
        for (int u = 0; u < kFoldBatch; ++u) {
          const int kk = kb + u < kHalf ? kb + u : kHalf - 1;
          const int src = (half * kHalf + kk) * 4;
          const int c0 = __builtin_amdgcn_ds_bpermute(src, cc0), c1 = __builtin_amdgcn_ds_bpermute(src, cc1);
          const int wl = __builtin_amdgcn_ds_bpermute(src, cwl), wh = __builtin_amdgcn_ds_bpermute(src, cwh);
          ww[u] = __longlong_as_double(((long long)wh << 32) | (unsigned)wl);
          cix[u] = kb + u < nmax && c0 + sub < c1 ? c0 + sub : -1;  // rows of C have <= 32 entries
          jj[u] = ld_i32(rFc, cix[u]);
        }
#pragma unroll
        for (int u = 0; u < kFoldBatch; ++u)
          if (cix[u] >= 0) {
            const int s = hash_find64(keys, jj[u]);
            if (s >= 0) unsafeAtomicAdd(g.F_out + cix[u], ww[u] * vals[s]);
          }
      }
    } else {
      // O(r,:) in its stored order
      const int o = h.o0 + sub < h.o1 ? h.o0 + sub : -1;
      const int c = ld_i32(rOc, o);
      if (o >= 0) {
        const int s = hash_find64(keys, c);
        g.O_val[o] = s >= 0 ? vals[s] : 0.0;
      }
    }
    wave_sync();
    if (h.o1 > h.o0) {
      keys[sub] = EMPTY;
      keys[sub + kHalf] = EMPTY;
      vals[sub] = 0.0;
      vals[sub + kHalf] = 0.0;
    }
    wave_sync();
  }
}

}  // namespace

bool rowmul_short_fits(const RowMulArgs& g) {
  return g.nnzX * 8 < (1LL << 31) && g.nnzY * 8 < (1LL << 31) && g.nnzO * 8 < (1LL << 31) &&
         ((long long)g.nX + 1) * 4 < (1LL << 31) && ((long long)g.nY + 1) * 4 < (1LL << 31) &&
         g.nnzF * 4 < (1LL << 31) && ((long long)g.nF + 1) * 4 < (1LL << 31);
}

static hipError_t launch_rowmul(const RowMulArgs& g, const int* rows, int count, bool long_x,
                                bool fold, int n_cu, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!rowmul_short_fits(g)) return hipErrorInvalidValue;
  // enough wavefronts for every CU to hold its full complement (32), each a contiguous run of
  // row pairs
  const long long npairs = ((long long)count + 1) / 2;
  const long long target = (long long)std::max(n_cu, 1) * 32;
  const int ppw = (int)std::max<long long>(1, (npairs + target - 1) / target);
  const long long waves = (npairs + ppw - 1) / ppw;
  const int grid = (int)((waves + kRmWaves - 1) / kRmWaves);
  const size_t lds = (size_t)kRmWaves * sizeof(HalfScratch);
  const dim3 gd(grid), bd(kRmWaves * WAVE);
  if (fold) {
    if (long_x)
      hipLaunchKernelGGL((k_rowmul_short<true, true>), gd, bd, lds, s, g, rows, count, ppw);
    else
      hipLaunchKernelGGL((k_rowmul_short<false, true>), gd, bd, lds, s, g, rows, count, ppw);
  } else {
    if (long_x)
      hipLaunchKernelGGL((k_rowmul_short<true, false>), gd, bd, lds, s, g, rows, count, ppw);
    else
      hipLaunchKernelGGL((k_rowmul_short<false, false>), gd, bd, lds, s, g, rows, count, ppw);
  }
  return hipGetLastError();
}

hipError_t launch_rowmul_short(const RowMulArgs& g, const int* rows, int count, bool long_x,
                               int n_cu, hipStream_t s) {
  return launch_rowmul(g, rows, count, long_x, false, n_cu, s);
}

hipError_t launch_atomic_fold_short(const RowMulArgs& g, const int* rows, int count, bool long_x,
                                    int n_cu, hipStream_t s) {
  return launch_rowmul(g, rows, count, long_x, true, n_cu, s);
}

}  // namespace ptapk
