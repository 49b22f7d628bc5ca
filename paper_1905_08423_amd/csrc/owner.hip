// Numeric all-at-once / merged product with the owner fold, short-row form.
//
// A workgroup of NW wavefronts owns a tile of rows of C (a compact set of rows chosen at symbolic
// time) whose values and column indices are held in LDS.  Each wavefront takes two fine rows I of the tile's list at a
// time, one per 32-lane half:
//   1. lane `sub` of the half loads A(I, a0+sub) and the extent of row J = A_col of P, then
//      loads every P(J, :) entry of that row at once and inserts A(I,J) * P(J,j) into the half's
//      hash map R_I (Alg. 3; compare-and-swap on the key, then an LDS FP64 add);
//   2. the entries P(I,i) with i in the tile (and in the pass's part, Alg. 8 / Alg. 10) are
//      compacted with a ballot;
//   3. for each such i the half walks C's row i in LDS, looks every column up in R_I and adds
//      P(I,i) * R_I(j) into the tile (Eq. allatonceoutproduct restricted to the owned rows).
// The tile is written to C once at the end.  Used when every fine row of the tile has at most
// 32 entries in A and in P and |R_I| <= 32; other tiles take the general kernel.  Consecutive
// row pairs of a wavefront are software-pipelined (see the loop).
#include "device.hpp"
#include "internal.hpp"

namespace ptapk {

namespace {
constexpr int kHalf = 32;
constexpr int kCap = 64;  // slots of one R_I table (|R_I| <= 32, load <= 1/2)
constexpr int kCapShift = 32 - 6;

struct HalfScratch {
  int keys[2][kCap];
  double vals[2][kCap];
  int sel_i[2][kHalf];
  double sel_w[2][kHalf];
};
}  // namespace

size_t owner_fast_wave_bytes() { return sizeof(HalfScratch); }

// Raw buffer resources: 32-bit byte offsets instead of 64-bit addresses, and one 8- or 16-byte
// load per lane for a pair of row pointers or four entries of a row of P.  (Each lane reads its
// own row of P, so the cost of a load is set by the number of distinct cache lines it touches:
// one wide load costs about what one 4-byte load costs.)
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
constexpr int kRawBufferFlags = 0x00020000;  // 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRawBufferFlags);
}
__device__ __forceinline__ v2u ld_pair(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, idx * 4, 0, 0);
}

// Per-lane state of one fine row at the successive stages of the pipelined loop (one row per
// 32-lane half; lane `sub` follows the row's A entry a0+sub and P entry p0+sub).
struct Stage2 {   // row extents known
  int I;          // fine row, or -1 past the end of the tile's list
  int t;          // a0 + sub if that A entry exists, else -1
  int e;          // p0 + sub if that P entry exists, else -1
};
struct Stage3 {   // column of this lane's A entry and of its P entry known
  int I, J, t, pi, e;  // J = column of A(I,t) (or -1); pi = column of P(I,e) (or -1)
};
struct Stage4 {   // extent of row J of P and the tile slot of column pi known
  int I, ps, pe, t, pi, e, sl;
};

__device__ __forceinline__ int st_header(const int* __restrict__ fine, int fr, int f1) {
  return fr < f1 ? fine[fr] : -1;
}
__device__ __forceinline__ Stage2 st_rows(int I, __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rP,
                                          int sub) {
  Stage2 r{I, -1, -1};
  if (I >= 0) {
    const v2u ar = ld_pair(rA, I), pr = ld_pair(rP, I);
    const int a0 = (int)ar[0], a1 = (int)ar[1], p0 = (int)pr[0], p1 = (int)pr[1];
    r.t = a0 + sub < a1 ? a0 + sub : -1;
    r.e = p0 + sub < p1 ? p0 + sub : -1;
  }
  return r;
}
__device__ __forceinline__ Stage3 st_entries(const Stage2& q, const Patterns& p) {
  Stage3 r{q.I, -1, q.t, -1, q.e};
  if (q.t >= 0) r.J = p.A_col[q.t];
  if (q.e >= 0) r.pi = p.P_col[q.e];
  return r;
}
__device__ __forceinline__ Stage4 st_pext(const Stage3& q, __amdgpu_buffer_rsrc_t rP,
                                          const int* __restrict__ slot) {
  Stage4 r{q.I, 0, 0, q.t, q.pi, q.e, -1};
  if (q.J >= 0) {
    const v2u pr = ld_pair(rP, q.J);
    r.ps = (int)pr[0];
    r.pe = (int)pr[1];
  }
  if (q.pi >= 0) r.sl = slot[q.pi];
  return r;
}

// Four consecutive entries k0..k0+3 of P: columns and values.  Wide loads when the whole
// window lies inside P's arrays; otherwise entry by entry up to `ke`.
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t rc, __amdgpu_buffer_rsrc_t rv,
                                      const int* __restrict__ P_col, const double* __restrict__ P_val,
                                      int k0, int ke, int nnzP, int (&jj)[4], double (&pv)[4]) {
  if (k0 + 4 <= nnzP) {
    const v4i c = __builtin_amdgcn_raw_buffer_load_b128(rc, k0 * 4, 0, 0);
    const v4i v01 = __builtin_amdgcn_raw_buffer_load_b128(rv, k0 * 8, 0, 0);
    const v4i v23 = __builtin_amdgcn_raw_buffer_load_b128(rv, k0 * 8 + 16, 0, 0);
    jj[0] = c[0];
    jj[1] = c[1];
    jj[2] = c[2];
    jj[3] = c[3];
    pv[0] = __hiloint2double(v01[1], v01[0]);
    pv[1] = __hiloint2double(v01[3], v01[2]);
    pv[2] = __hiloint2double(v23[1], v23[0]);
    pv[3] = __hiloint2double(v23[3], v23[2]);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      jj[u] = 0;
      pv[u] = 0.0;
      if (k0 + u < ke) {
        jj[u] = P_col[k0 + u];
        pv[u] = P_val[k0 + u];
      }
    }
  }
}

__device__ __forceinline__ void hash_add64(int* keys, double* vals, int key, double v) {
  unsigned s = hslot(key, kCapShift);
  while (true) {
    const int old = atomicCAS(keys + s, EMPTY, key);
    if (old == EMPTY || old == key) break;
    s = (s + 1) & (kCap - 1);
  }
  atomicAdd(vals + s, v);
}

// One tile of the owner fold by the whole workgroup (NW wavefronts); smem holds the tile and the
// per-wavefront hash tables.  Ends with the tile written to C and a workgroup barrier.
template <int NW>
__device__ __forceinline__ void owner_fast_tile(const NumericArgs& a, int tile, const TileSet& ts,
                                                const int* __restrict__ tile_fptr,
                                                const int* __restrict__ tile_fine, int TE,
                                                unsigned char* smem) {
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int half = ln / kHalf, sub = ln % kHalf;
  const int tp = ts.ptr[tile], nr = ts.ptr[tile + 1] - tp;
  const Patterns& p = a.p;

  double* tv = reinterpret_cast<double*>(smem);
  int* tc = reinterpret_cast<int*>(smem + (size_t)TE * sizeof(double));
  int* trp = tc + TE;
  HalfScratch* hs = reinterpret_cast<HalfScratch*>(
                        smem + (((size_t)TE * 12 + ((size_t)kTileRows + 1) * 4 + 15) / 16) * 16) +
                    wid;
  tile_load(ts.rows, tp, nr, a.C_rowptr, a.C_col, trp, tc, tv);
  int* keys = hs->keys[half];
  double* vals = hs->vals[half];
  keys[sub] = EMPTY;
  keys[sub + kHalf] = EMPTY;
  vals[sub] = 0.0;
  vals[sub + kHalf] = 0.0;
  __syncthreads();

  const int f0 = tile_fptr[tile], f1 = tile_fptr[tile + 1];
  const int step = 2 * NW;
  const int nnzP = p.P_rowptr[p.n];
  const __amdgpu_buffer_rsrc_t rA = buffer_rsrc(p.A_rowptr, (unsigned)(p.n + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rP = buffer_rsrc(p.P_rowptr, (unsigned)(p.n + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rPc = buffer_rsrc(p.P_col, (unsigned)nnzP * 4u);
  const __amdgpu_buffer_rsrc_t rPv = buffer_rsrc(a.P_val, (unsigned)nnzP * 8u);
  const int npass = a.part < 0 ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int part = a.part < 0 ? (pass == 0 ? PART_OFF : PART_ON) : a.part;
    // Software pipeline over the wavefront's row pairs f, f+step, f+2*step, ...: while the
    // pair being folded (cur) works in LDS, the next pairs advance one load stage each (row
    // index -> row extents -> entries of A and P -> extent of the row of P), so each dependent
    // load overlaps one iteration of LDS work instead of stalling the wavefront.
    const int fb = f0 + 2 * wid + half;
    Stage4 cur = st_pext(st_entries(st_rows(st_header(tile_fine, fb, f1), rA, rP, sub), p), rP, ts.slot);
    Stage3 nxt = st_entries(st_rows(st_header(tile_fine, fb + step, f1), rA, rP, sub), p);
    Stage2 nn = st_rows(st_header(tile_fine, fb + 2 * step, f1), rA, rP, sub);
    for (int f = f0 + 2 * wid; f < f1; f += step) {
      // (1) values of cur's A and P entries and its first four products (the rest load in (4))
      const double cav = cur.t >= 0 ? a.A_val[cur.t] : 0.0;
      const double cpw = cur.e >= 0 ? a.P_val[cur.e] : 0.0;
      int jj[4];
      double pv[4];
      load4(rPc, rPv, p.P_col, a.P_val, cur.ps, cur.pe, nnzP, jj, pv);
      // (2) one load stage for each following pair
      const Stage4 nxt4 = st_pext(nxt, rP, ts.slot);
      const Stage3 nn3 = st_entries(nn, p);
      const Stage2 nnn2 = st_rows(st_header(tile_fine, f + 3 * step + half, f1), rA, rP, sub);
      // (3) owned entries of P(I,:) of cur, compacted per half
      const bool in_t = cur.sl >= 0 && (cur.sl >> kTileRowBits) == tile &&
                        part_takes(part, cur.I, cur.pi, p.n, p.m, a.K);
      const unsigned long long bal = ballot(in_t);
      const unsigned hm = half ? (unsigned)(bal >> 32) : (unsigned)bal;
      const int nsel = __popc(hm);
      if (in_t) {
        const int pos = __popc(hm & ((1u << sub) - 1u));
        hs->sel_i[half][pos] = cur.sl & (kTileRows - 1);
        hs->sel_w[half][pos] = cpw;
      }
      const int nmax = max(nsel, __shfl_xor(nsel, kHalf, WAVE));
      // (4) R_I of cur in the half's hash map
      if (nsel > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (cur.ps + u < cur.pe) hash_add64(keys, vals, jj[u], cav * pv[u]);
        for (int k0 = cur.ps + 4; k0 < cur.pe; k0 += 4) {
          load4(rPc, rPv, p.P_col, a.P_val, k0, cur.pe, nnzP, jj, pv);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (k0 + u < cur.pe) hash_add64(keys, vals, jj[u], cav * pv[u]);
        }
      }
      wave_sync();
      // (6) fold the owned part of P(I,:) (x) R_I into the tile
      for (int kk = 0; kk < nmax; ++kk) {
        if (kk < nsel) {
          const int rl = hs->sel_i[half][kk];
          const double wk = hs->sel_w[half][kk];
          const int ce = trp[rl + 1];
          for (int c = trp[rl] + sub; c < ce; c += kHalf) {
            const int j = tc[c];
            unsigned s = hslot(j, kCapShift);
            int kf;
            while ((kf = keys[s]) != j && kf != EMPTY) s = (s + 1) & (kCap - 1);
            if (kf == j) atomicAdd(tv + c, wk * vals[s]);
          }
        }
      }
      wave_sync();
      if (nsel > 0) {
        keys[sub] = EMPTY;
        keys[sub + kHalf] = EMPTY;
        vals[sub] = 0.0;
        vals[sub + kHalf] = 0.0;
      }
      wave_sync();
      cur = nxt4;
      nxt = nn3;
      nn = nnn2;
    }
  }
  __syncthreads();
  tile_store(ts.rows, tp, nr, a.C_rowptr, trp, tv, a.C_val);
  __syncthreads();
}

template <int NW>
__global__ __launch_bounds__(NW * WAVE, 8) void k_owner_fast(NumericArgs a, const int* __restrict__ tiles,
                                                             TileSet ts,
                                                             const int* __restrict__ tile_fptr,
                                                             const int* __restrict__ tile_fine, int TE,
                                                             int xcd_remap) {
  extern __shared__ __align__(16) unsigned char smem[];
  int b = blockIdx.x;
  if (xcd_remap) {
    // Workgroups are dispatched to the 8 XCDs round-robin; give XCD x a contiguous run of tiles
    // so neighbouring tiles (which share fine rows) meet in the same L2.
    const int T = gridDim.x, q = T / 8, rem = T % 8, x = b % 8, k = b / 8;
    b = x * q + min(x, rem) + k;
  }
  owner_fast_tile<NW>(a, tiles[b], ts, tile_fptr, tile_fine, TE, smem);
}

// Batched form: a persistent grid works through a list of (plan, tile) items, every item one tile
// of one plan's owner fold.  The list (plan by plan, tiles in order) is cut into 8 contiguous
// chunks with a counter each; the workgroups of XCD x (workgroups are dispatched to the XCDs
// round-robin) take items from chunk x, so neighbouring tiles share that XCD's L2, and then help
// with the other chunks.
template <int NW>
__global__ __launch_bounds__(NW * WAVE, 8) void k_owner_fast_batch(const OwnerBatchPlan* __restrict__ plans,
                                                                   const int2* __restrict__ items,
                                                                   int nitems, int* counters) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int next;
  const int xcd = blockIdx.x % kXcds;
  for (int c = 0; c < kXcds; ++c) {
    const int x = (xcd + c) % kXcds;
    const int hi = (int)(((long long)(x + 1) * nitems) / kXcds);
    const int lo = (int)(((long long)x * nitems) / kXcds);
    while (true) {
      if (threadIdx.x == 0) next = lo + atomicAdd(counters + x, 1);
      __syncthreads();
      // the item is the same for the whole workgroup: read it into scalar registers, so the
      // plan's pointers are loaded with scalar loads and stay out of the vector registers
      const int it = __builtin_amdgcn_readfirstlane(next);
      __syncthreads();
      if (it >= hi) break;
      const int2 w = items[it];
      const int pk = __builtin_amdgcn_readfirstlane(w.x);
      const int tl = __builtin_amdgcn_readfirstlane(w.y);
      const OwnerBatchPlan& pl = plans[pk];
      owner_fast_tile<NW>(pl.a, tl, pl.ts, pl.tile_fptr, pl.tile_fine, pl.TE, smem);
    }
  }
}

size_t owner_fast_lds_bytes(int TE, int nw) {
  return (((size_t)TE * 12 + ((size_t)kTileRows + 1) * 4 + 15) / 16) * 16 + (size_t)nw * sizeof(HalfScratch);
}

hipError_t launch_owner_fast(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                             const int* tile_fptr, const int* tile_fine, int TE, int nw,
                             bool xcd_remap, hipStream_t s) {
  if (tc.count == 0) return hipSuccess;
  const size_t lds = owner_fast_lds_bytes(TE, nw);
  const int remap = xcd_remap ? 1 : 0;
  if (nw == 16) {
    hipLaunchKernelGGL(k_owner_fast<16>, dim3(tc.count), dim3(16 * WAVE), lds, s, a, tc.tiles,
                       ts, tile_fptr, tile_fine, TE, remap);
  } else if (nw == 8) {
    hipLaunchKernelGGL(k_owner_fast<8>, dim3(tc.count), dim3(8 * WAVE), lds, s, a, tc.tiles,
                       ts, tile_fptr, tile_fine, TE, remap);
  } else {
    hipLaunchKernelGGL(k_owner_fast<4>, dim3(tc.count), dim3(4 * WAVE), lds, s, a, tc.tiles,
                       ts, tile_fptr, tile_fine, TE, remap);
  }
  return hipGetLastError();
}

hipError_t launch_owner_fast_batch(const OwnerBatchPlan* plans, const int2* items, int nitems,
                                   int* counter, int grid, size_t lds, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner_fast_batch<kFastWaves>, dim3(grid), dim3(kFastWaves * WAVE), lds, s,
                     plans, items, nitems, counter);
  return hipGetLastError();
}

}  // namespace ptapk
