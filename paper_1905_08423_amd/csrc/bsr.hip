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
// Blocks are read one entry per lane (the wavefront's load is contiguous); a lane takes the
// other entries of its column from the lanes holding them (ds_bpermute), which costs the
// address unit a quarter of loading the column in every lane.
// 4 x 4 blocks take k_bsr_flat4 instead, which forms the blocks U of up to 32 entries of A(I,:)
// first and then deals the row's block products out 32 at a time (see there).
// The C pattern is the structural block product computed by the scalar symbolic phase on the
// block patterns.  Summation order varies between runs (LDS and device atomics).
#include "device.hpp"
#include "internal.hpp"
#include "short_rows.hpp"

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
constexpr int kU = 4;  // products of a step whose loads are issued together

// 4 x 4 blocks: a group of 16 lanes is one DPP row, block row r is quad r.  Rotating the row by
// 4d lanes brings entry ((r - d) mod 4, c) to lane (r, c), so a column of a block is gathered
// with three rotations, and row r of a block with four quad broadcasts, all in VALU.
template <int CTRL>
__device__ __forceinline__ double dpp_dbl(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kRor4 = 0x124, kRor8 = 0x128, kRor12 = 0x12C;  // row_ror:4, :8, :12
// sum_k w[k] X[k][c] for lane (r, c), with wr[d] = w[(r - d) mod 4] precomputed
__device__ __forceinline__ double col_dot4(const double (&wr)[4], double x) {
  return wr[0] * x + wr[1] * dpp_dbl<kRor4>(x) + wr[2] * dpp_dbl<kRor8>(x) + wr[3] * dpp_dbl<kRor12>(x);
}
// w[(r - d) mod 4] for d = 0..3 from the lane's w[0..3]
__device__ __forceinline__ void rot_coef4(const double (&w)[4], int r, double (&wr)[4]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int k = (r - d) & 3;
    wr[d] = k == 0 ? w[0] : k == 1 ? w[1] : k == 2 ? w[2] : w[3];
  }
}

// One step of row I for this lane's group: its entry A(I,J) (this lane's element) and the
// extent of row J of P.
struct StepLoad {
  double own;
  int ps, pe;
  bool ok;
};
template <int B2, int G>
__device__ __forceinline__ StepLoad step_load(const BsrArgs& a, int t0, int a1, int g, int ent, bool in_group) {
  const int t = t0 + g;
  StepLoad r{0.0, 0, 0, in_group && t < a1};
  if (r.ok) {
    const int J = a.A_col[t];
    r.own = a.A_val[(size_t)t * B2 + ent];
    r.ps = a.P_rowptr[J];
    r.pe = a.P_rowptr[J + 1];
  }
  return r;
}
}  // namespace

// LDS layout of the row kernel: keys[cap] (int), pos[cap] (int), then (LDS accumulation only)
// acc[ncmax * bs^2] (double, 16-byte aligned).
// The 4 x 4 kernel adds one FlatScratch per wavefront after them.
namespace {
constexpr int kFlatSeg = 32;    // entries of A(I,:) whose blocks U are staged at a time
constexpr int kFlatRounds = 8;  // rounds of 4 block products whose loads are issued together
constexpr int kFlatWin = 4 * kFlatRounds;  // products dealt per batch
static_assert(kFlatWin <= 32, "a batch's products are numbered by the lanes of one half");
struct FlatScratch {
  double urot[kFlatSeg][16];  // U = P(I,i)^T A(I,J) of each staged entry, row r rotated (below)
  int2 rec[kFlatSeg];         // nonempty segments of the walk by rank: (offset into P, entry)
};
__host__ __device__ inline size_t bsr_head_bytes(int bs, int cap, int ncmax, bool lds_acc) {
  const size_t head = (((size_t)cap * 8) + 15) / 16 * 16;
  return lds_acc ? head + (size_t)ncmax * bs * bs * sizeof(double) : head;
}
}  // namespace

size_t bsr_lds_bytes(int bs, int cap, int ncmax, bool lds_acc) {
  const size_t head = (bsr_head_bytes(bs, cap, ncmax, lds_acc) + 15) / 16 * 16;
  return bs == 4 ? head + kBsrWaves * sizeof(FlatScratch) : head;
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
    // step loads (the entry A(I,J) of this lane's group, the extent of row J of P) are issued
    // one step ahead; the products of a step issue their loads kU at a time
    StepLoad nx = step_load<B2, G>(a, a0, a1, g, ent, in_group);
    for (int t0 = a0; t0 < a1; t0 += G) {
      const StepLoad cu = nx;
      if (t0 + G < a1) nx = step_load<B2, G>(a, t0 + G, a1, g, ent, in_group);
      double U = 0.0;
      double Ur[BS];  // row r of this group's U
#pragma unroll
      for (int k = 0; k < BS; ++k) U += T[k] * lane_dbl(cu.own, in_group ? g * B2 + k * BS + c : ln);
#pragma unroll
      for (int k = 0; k < BS; ++k) Ur[k] = lane_dbl(U, in_group ? g * B2 + r * BS + k : ln);
      const int len = cu.pe - cu.ps;
      const int lmax = wave_max(len);
      for (int u0 = 0; u0 < lmax; u0 += kU) {
        double pown[kU];
        int jj[kU];
#pragma unroll
        for (int v = 0; v < kU; ++v) {
          const bool live = cu.ok && u0 + v < len;
          const int e2 = cu.ps + u0 + v;
          pown[v] = live ? a.P_val[(size_t)e2 * B2 + ent] : 0.0;
          jj[v] = live ? a.P_col[e2] : -1;
        }
#pragma unroll
        for (int v = 0; v < kU; ++v) {
          if (u0 + v >= lmax) break;
          double V = 0.0;
#pragma unroll
          for (int k = 0; k < BS; ++k) V += Ur[k] * lane_dbl(pown[v], in_group ? g * B2 + k * BS + c : ln);
          const int j = jj[v];
          if (j >= 0) {
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
  }
  if (LDS_ACC) {
    __syncthreads();
    for (int x = threadIdx.x; x < nc * B2; x += blockDim.x) a.C_val[(size_t)c0 * B2 + x] = acc[x];
  }
}


// 4 x 4 blocks by a flattened walk.  The products of row I are the pairs (entry J of A(I,:),
// block P(J,j)); taken entry by entry, every round of four products waits for its loads of P
// before it can start.  Here a wavefront first forms U_J = P(I,i)^T A(I,J) for up to kFlatSeg
// entries of A(I,:) (group g of 16 lanes takes entries g, g+4, ...; lane (r, c) holds U_J[r][c])
// and leaves them in LDS, then deals the products of those entries out 32 at a time (a prefix
// sum of the lengths of the rows of P gives every product its entry and its block of P), so the
// loads of 32 block products are in flight together.  Lane (r, c) of the group that takes a
// product P(J,j) adds sum_k U_J[r][k] P(J,j)[k][c] into block j of row i of C.  U_J is stored
// with row r rotated, urot[J][4r + d] = U_J[r][(r - d) mod 4], which is the order in which
// col_dot4 takes the coefficients, so a lane reads its four with two 16-byte LDS loads.
template <bool LDS_ACC>
__global__ __launch_bounds__(kBsrWaves * WAVE) void k_bsr_flat4(BsrArgs a, const int* __restrict__ rows,
                                                                int nrows, int cap, int ncmax, int xcd_remap) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* keys = reinterpret_cast<int*>(smem);
  int* pos = keys + cap;
  double* acc = reinterpret_cast<double*>(smem + (((size_t)cap * 8) + 15) / 16 * 16);
  const int ln = lane(), wid = threadIdx.x / WAVE;
  FlatScratch* fs = reinterpret_cast<FlatScratch*>(
                        smem + (bsr_head_bytes(4, cap, ncmax, LDS_ACC) + 15) / 16 * 16) + wid;
  const int g = ln >> 4, ent = ln & 15, r = ent >> 2, c = ent & 3;
  const int q32 = ln & 31;
  const unsigned shift = 32u - (unsigned)__builtin_ctz((unsigned)cap);

  int b = blockIdx.x;
  if (xcd_remap) {
    const int T = gridDim.x, q = T / 8, rem = T % 8, x = b % 8, k = b / 8;
    b = x * q + min(x, rem) + k;
  }
  if (b >= nrows) return;
  const int i = rows[b];
  const int c0 = a.C_rowptr[i], nc = a.C_rowptr[i + 1] - c0;

  if (LDS_ACC) {
    for (int s = threadIdx.x; s < cap; s += blockDim.x) keys[s] = EMPTY;
    for (int x = threadIdx.x; x < nc * 16; x += blockDim.x) acc[x] = 0.0;
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
    const size_t pIi = (size_t)a.pt_pos[qq] * 16;
    double T[4];  // lane (r, c): column r of P(I,i), i.e. row r of P(I,i)^T
#pragma unroll
    for (int k = 0; k < 4; ++k) T[k] = a.P_val[pIi + k * 4 + r];
    double Tr[4];
    rot_coef4(T, r, Tr);
    const int a0 = a.A_rowptr[I], a1 = a.A_rowptr[I + 1];
    for (int ch = a0; ch < a1; ch += kFlatSeg) {
      const int ne = min(kFlatSeg, a1 - ch);
      // lane q < ne of the lower half: entry ch + q and the extent of its row of P
      int ps = 0, len = 0;
      if (ln < ne) {
        const int J = a.A_col[ch + ln];
        ps = a.P_rowptr[J];
        len = a.P_rowptr[J + 1] - ps;
      }
      double own[kFlatSeg / 4];
#pragma unroll
      for (int s = 0; s < kFlatSeg / 4; ++s) {
        const int q = 4 * s + g;
        own[s] = q < ne ? a.A_val[(size_t)(ch + q) * 16 + ent] : 0.0;
      }
      const int incl = half_incl_scan(len);  // upper half: len 0
      const int tot = __builtin_amdgcn_readlane(incl, 31);
      const unsigned long long nonempty = ballot(len > 0);
      if (len > 0) fs->rec[prefix_count(nonempty)] = make_int2(ps - (incl - len), ln);
#pragma unroll
      for (int s = 0; s < kFlatSeg / 4; ++s) {
        if (4 * s < ne) {  // uniform: every lane takes part in the row rotations
          const double U = col_dot4(Tr, own[s]);
          if (4 * s + g < ne) fs->urot[4 * s + g][4 * r + ((r - c) & 3)] = U;
        }
      }
      wave_sync();
      int before = 0;  // nonempty segments that end before the current window
      for (int b0 = 0; b0 < tot; b0 += kFlatWin) {
        // lane p < kFlatWin (of each half): product b0 + p, its segment by rank and its block of
        // P; the window's segment ends are counted only up to kFlatWin, so `before` stays the
        // rank of the segment that holds product b0 of the next batch
        const int d = incl - b0 - 1;
        const int bit = (len > 0 && (unsigned)d < (unsigned)kFlatWin) ? (int)(1u << d) : 0;
        const unsigned ends = (unsigned)__builtin_amdgcn_readlane(half_or_scan(bit), 31);
        const int rk = (before + __popc(ends & ((1u << q32) - 1u))) & (kFlatSeg - 1);
        const int2 rc = fs->rec[rk];
        // positions past the batch or the chunk's products deal nothing: their rank may name a
        // record not written for this chunk, so neither its offset nor its entry is used
        const int e_p = q32 < kFlatWin && b0 + q32 < tot ? b0 + q32 + rc.x : -1;
        const int t_p = e_p >= 0 ? rc.y : 0;
        before += __popc(ends);
        // round u: group g takes product 4u + g
        int eu[kFlatRounds], tu[kFlatRounds], jj[kFlatRounds];
        double pv[kFlatRounds];
#pragma unroll
        for (int u = 0; u < kFlatRounds; ++u) {
          eu[u] = __builtin_amdgcn_ds_bpermute((4 * u + g) * 4, e_p);
          tu[u] = __builtin_amdgcn_ds_bpermute((4 * u + g) * 4, t_p);
        }
#pragma unroll
        for (int u = 0; u < kFlatRounds; ++u) {
          pv[u] = eu[u] >= 0 ? a.P_val[(size_t)eu[u] * 16 + ent] : 0.0;
          jj[u] = eu[u] >= 0 ? a.P_col[eu[u]] : -1;
        }
        const int nr = min(kFlatRounds, (tot - b0 + 3) / 4);
#pragma unroll
        for (int u = 0; u < kFlatRounds; ++u) {
          if (u < nr) {  // uniform
            const double2* ur = reinterpret_cast<const double2*>(&fs->urot[tu[u]][4 * r]);
            const double2 u01 = ur[0], u23 = ur[1];
            const double w[4] = {u01.x, u01.y, u23.x, u23.y};
            const double V = col_dot4(w, pv[u]);
            const int j = jj[u];
            if (j >= 0) {
              if (LDS_ACC) {
                unsigned s = hslot(j, (int)shift);
                for (int it = 1; keys[s] != j && it < cap; ++it) s = (s + 1) & (unsigned)(cap - 1);
                if (keys[s] == j) atomicAdd(acc + (size_t)pos[s] * 16 + ent, V);
              } else {
                const int p = row_find(a.C_col, c0, nc, j);
                atomicAdd(a.C_val + ((size_t)c0 + p) * 16 + ent, V);
              }
            }
          }
        }
      }
      wave_sync();  // the staged blocks and records are rewritten by the next chunk
    }
  }
  if (LDS_ACC) {
    __syncthreads();
    for (int x = threadIdx.x; x < nc * 16; x += blockDim.x) a.C_val[(size_t)c0 * 16 + x] = acc[x];
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
    case 4: {
      const size_t lds = bsr_lds_bytes(4, cap, ncmax, lds_acc);
      if (lds_acc)
        hipLaunchKernelGGL(k_bsr_flat4<true>, dim3(nrows), dim3(kBsrWaves * WAVE), lds, s, a, rows, nrows, cap,
                           ncmax, remap ? 1 : 0);
      else
        hipLaunchKernelGGL(k_bsr_flat4<false>, dim3(nrows), dim3(kBsrWaves * WAVE), lds, s, a, rows, nrows, cap,
                           ncmax, remap ? 1 : 0);
      break;
    }
    case 5: launch_bs<5>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 6: launch_bs<6>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 7: launch_bs<7>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    case 8: launch_bs<8>(a, rows, nrows, cap, ncmax, lds_acc, remap, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ptapk
