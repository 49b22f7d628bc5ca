// Numeric C = P^T A P for block-sparse A and P (BSR: dense bs x bs blocks, row-major, on a
// block pattern), in the row form of Eq. allatoncerow:
//   C(i,:) = sum over the fine block rows I with P(I,i) stored of  P(I,i)^T A(I,:) P.
// A workgroup owns a row i of C.  Its block columns are entered in an LDS hash (column ->
// position in the row) and its blocks are accumulated in LDS (or, for rows too long for LDS,
// in C itself with device-wide FP64 atomics).  The workgroup's wavefronts take the fine rows I
// of column i of P in turn; in a wavefront the 64 lanes form 64 / bs^2 groups of bs^2 lanes,
// lane (r, c) of group g holding entry (r, c) of one block:
//   1. group g takes the entry A(I,J) of step t0 + g of row I and forms U = P(I,i)^T A(I,J)
//      (lane (r,c): sum_k P(I,i)[k][r] A(I,J)[k][c]);
//   2. every lane fetches row r of its group's U from the lanes holding it (ds_bpermute);
//   3. for each entry P(J,j) of row J of P the lane adds sum_k U[r][k] P(J,j)[k][c] into block
//      j of row i of C (LDS FP64 add at the block's position).
// The C pattern is the structural block product computed by the scalar symbolic phase on the
// block patterns.  Summation order varies between runs (LDS and device atomics).
#include "device.hpp"
#include "internal.hpp"

namespace ptapk {

namespace {
constexpr int kBsrWaves = 4;  // wavefronts per workgroup

// The value of `v` in lane `src` (every lane of the wavefront active).
__device__ __forceinline__ double lane_dbl(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src * 4, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src * 4, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Position of column j in the sorted row C_col[c0 .. c0 + nc) (present by construction of the
// pattern); binary search in device memory, for rows whose table does not fit in LDS.
__device__ __forceinline__ int row_find(const int* __restrict__ col, int c0, int nc, int j) {
  int lo = 0, hi = nc;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (col[c0 + mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}
}  // namespace

// LDS layout of the row kernel: keys[cap] (int), pos[cap] (int), then (LDS accumulation only)
// acc[ncmax * bs^2] (double, 16-byte aligned).
size_t bsr_lds_bytes(int bs, int cap, int ncmax, bool lds_acc) {
  const size_t head = (((size_t)cap * 8) + 15) / 16 * 16;
  return lds_acc ? head + (size_t)ncmax * bs * bs * sizeof(double) : head;
}

template <int BS, bool LDS_ACC>
__global__ __launch_bounds__(kBsrWaves * WAVE) void k_bsr_numeric(BsrArgs a, const int* __restrict__ rows,
                                                                  int nrows, int cap, int xcd_remap) {
  constexpr int B2 = BS * BS;
  constexpr int G = WAVE / B2;  // block products per wavefront step
  extern __shared__ __align__(16) unsigned char smem[];
  int* keys = reinterpret_cast<int*>(smem);
  int* pos = keys + cap;
  double* acc = reinterpret_cast<double*>(smem + (((size_t)cap * 8) + 15) / 16 * 16);
  const int ln = lane(), wid = threadIdx.x / WAVE;
  const int g = ln / B2, ent = ln % B2, r = ent / BS, c = ent % BS;
  const bool in_group = g < G;
  const unsigned shift = 32u - (unsigned)__builtin_ctz((unsigned)cap);

  int b = blockIdx.x;
  if (xcd_remap) {
    // workgroups are dispatched to the 8 XCDs round-robin: give each XCD a contiguous run of
    // rows of C, whose fine rows overlap, so that they meet in the same L2
    const int T = gridDim.x, q = T / 8, rem = T % 8, x = b % 8, k = b / 8;
    b = x * q + min(x, rem) + k;
  }
  if (b >= nrows) return;
  const int i = rows[b];
  const int c0 = a.C_rowptr[i], nc = a.C_rowptr[i + 1] - c0;

  // the row's columns -> positions (LDS hash), accumulators cleared
  if (LDS_ACC) {
    for (int s = threadIdx.x; s < cap; s += blockDim.x) keys[s] = EMPTY;
    for (int x = threadIdx.x; x < nc * B2; x += blockDim.x) acc[x] = 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q < nc; q += blockDim.x) {
      const int j = a.C_col[c0 + q];
      unsigned s = hslot(j, (int)shift);
      for (int it = 0; it < cap && atomicCAS(keys + s, EMPTY, j) != EMPTY; ++it) s = (s + 1) & (unsigned)(cap - 1);
      pos[s] = q;
    }
    __syncthreads();
  }

  for (int qq = a.pt_ptr[i] + wid; qq < a.pt_ptr[i + 1]; qq += kBsrWaves) {
    const int I = a.pt_row[qq];
    const size_t pIi = (size_t)a.pt_pos[qq] * B2;
    double T[BS];  // lane (r, c): row r of P(I,i)^T, i.e. column r of P(I,i)
#pragma unroll
    for (int k = 0; k < BS; ++k) T[k] = a.P_val[pIi + k * BS + r];
    const int a0 = a.A_rowptr[I], a1 = a.A_rowptr[I + 1];
    for (int t0 = a0; t0 < a1; t0 += G) {
      const int t = t0 + g;
      const bool ok = in_group && t < a1;
      double U = 0.0;
      int ps = 0, pe = 0;
      if (ok) {
        const int J = a.A_col[t];
        const double* __restrict__ Ab = a.A_val + (size_t)t * B2;
#pragma unroll
        for (int k = 0; k < BS; ++k) U += T[k] * Ab[k * BS + c];
        ps = a.P_rowptr[J];
        pe = a.P_rowptr[J + 1];
      }
      double Ur[BS];  // row r of this group's U
#pragma unroll
      for (int k = 0; k < BS; ++k) Ur[k] = lane_dbl(U, in_group ? g * B2 + r * BS + k : ln);
      const int len = pe - ps;
      const int lmax = wave_max(len);
      for (int u = 0; u < lmax; ++u) {
        if (ok && u < len) {
          const int e2 = ps + u;
          const int j = a.P_col[e2];
          const double* __restrict__ Pb = a.P_val + (size_t)e2 * B2;
          double V = 0.0;
#pragma unroll
          for (int k = 0; k < BS; ++k) V += Ur[k] * Pb[k * BS + c];
          if (LDS_ACC) {
            // j is a column of row i by construction of the pattern; the probe is bounded anyway
            unsigned s = hslot(j, (int)shift);
            for (int it = 1; keys[s] != j && it < cap; ++it) s = (s + 1) & (unsigned)(cap - 1);
            if (keys[s] == j) atomicAdd(acc + (size_t)pos[s] * B2 + ent, V);
          } else {
            const int p = row_find(a.C_col, c0, nc, j);
            atomicAdd(a.C_val + ((size_t)c0 + p) * B2 + ent, V);
          }
        }
      }
    }
  }
  if (LDS_ACC) {
    __syncthreads();
    for (int x = threadIdx.x; x < nc * B2; x += blockDim.x) a.C_val[(size_t)c0 * B2 + x] = acc[x];
  }
}

template <int BS>
static void launch_bs(const BsrArgs& a, const int* rows, int nrows, int cap, int ncmax, bool lds_acc,
                      bool remap, hipStream_t s) {
  const size_t lds = bsr_lds_bytes(BS, cap, ncmax, lds_acc);
  if (lds_acc)
    hipLaunchKernelGGL((k_bsr_numeric<BS, true>), dim3(nrows), dim3(kBsrWaves * WAVE), lds, s, a, rows, nrows,
                       cap, remap ? 1 : 0);
  else
    hipLaunchKernelGGL((k_bsr_numeric<BS, false>), dim3(nrows), dim3(kBsrWaves * WAVE), lds, s, a, rows, nrows,
                       cap, remap ? 1 : 0);
}

hipError_t launch_bsr_numeric(const BsrArgs& a, int bs, const int* rows, int nrows, int cap, int ncmax,
                              bool lds_acc, bool remap, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  switch (bs) {
    case 1: launch_bs<1>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 2: launch_bs<2>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 3: launch_bs<3>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 4: launch_bs<4>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 5: launch_bs<5>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 6: launch_bs<6>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 7: launch_bs<7>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 8: launch_bs<8>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ptapk
