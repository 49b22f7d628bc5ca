// Numeric all-at-once / merged product with the owner fold, short-row form.
//
// A workgroup of NW wavefronts owns a tile of rows of C (a compact set of rows chosen at symbolic
// time) whose values and column indices are held in LDS.  Each wavefront takes two fine rows I of
// the tile's list at a time, one per 32-lane half:
//   1. lane `sub` of the half holds A(I, a0+sub), the extent of row J = A_col of P and P(I, p0+sub);
//   2. the products A(I,J) * P(J,j) of the row are dealt out 32 at a time over the half's lanes
//      (a prefix sum of the lengths of the rows of P gives every lane its product and its row J),
//      so consecutive lanes read consecutive entries of P, and each product is added into the
//      half's hash map R_I (Alg. 3; compare-and-swap on the key, then an LDS FP64 add);
//   3. for each entry P(I,i) with i in the tile (and in the pass's part, Alg. 8 / Alg. 10) the
//      half walks C's row i in LDS, looks every column up in R_I and adds P(I,i) * R_I(j) into
//      the tile (Eq. allatonceoutproduct restricted to the owned rows).
// The tile is written to C once at the end.  Used when every fine row of the tile has at most
// 32 entries in A and in P and |R_I| <= 32; other tiles take the general kernel.  Consecutive
// row pairs of a wavefront are software-pipelined (see the loop).
#include "device.hpp"
#include "internal.hpp"
#include "short_rows.hpp"

namespace ptapk {

namespace {
constexpr int kPrefetch = 4;  // product-walk steps whose loads are issued together
}  // namespace

size_t owner_fast_wave_bytes() { return sizeof(HalfScratch); }

// Per-lane state of one fine row at the successive stages of the pipelined loop (one row per
// 32-lane half; lane `sub` follows the row's A entry a0+sub and P entry p0+sub).
struct Stage2 {   // row index and extents (the same in every lane of a half)
  int I;          // fine row, or -1 past the end of the tile's list
  int a0, a1, p0, p1;
};
struct Stage3 {   // column of this lane's A entry and of its P entry known
  int I, J, t, pi, e;  // t = a0+sub, e = p0+sub (or -1); J = A_col[t] (with the numeric cache:
                       // the packed extent of row J of P), pi = P_col[e] (or -1)
};
struct Stage4 {   // extent of row J of P, the tile slot of column pi and both values known
  int I, ps, pe, t, pi, e, sl;
  double av, pw;  // A(I,J) and P(I,pi) (0 where the entry does not exist)
};

// Row headers of a wavefront's next 32 row pairs: lane h*32 + k holds the fine row of iteration
// it0 + k of half h and that row's extents in A and P.  They are loaded together once per 32
// iterations, so the dependent loads row index -> row pointers wait once per block instead of in
// every iteration (a wait on a vector load also waits for every load issued before it).
__device__ __forceinline__ Stage2 hdr_load(const int* __restrict__ fine, int fr, int f1,
                                           __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rP) {
  Stage2 r{-1, 0, 0, 0, 0};
  if (fr < f1) {
    r.I = fine[fr];
    const v2u ar = ld_pair(rA, r.I), pr = ld_pair(rP, r.I);
    r.a0 = (int)ar[0];
    r.a1 = (int)ar[1];
    r.p0 = (int)pr[0];
    r.p1 = (int)pr[1];
  }
  return r;
}
// The header of iteration it0 + k for this lane's half (k uniform): a backward permute from
// lane half*32 + k (one LDS-crossbar operation per value instead of two readlanes and a select).
// Every lane of the wavefront must be active.
__device__ __forceinline__ Stage2 hdr_get(const Stage2& b, int k, int half) {
  const int src = (half * kHalf + k) * 4;
  Stage2 r;
  r.I = __builtin_amdgcn_ds_bpermute(src, b.I);
  r.a0 = __builtin_amdgcn_ds_bpermute(src, b.a0);
  r.a1 = __builtin_amdgcn_ds_bpermute(src, b.a1);
  r.p0 = __builtin_amdgcn_ds_bpermute(src, b.p0);
  r.p1 = __builtin_amdgcn_ds_bpermute(src, b.p1);
  return r;
}

// Buffer resources of the arrays the kernel gathers from.  Every gather below is issued
// unconditionally: an invalid entry passes index -1, whose byte offset lies past the end of the
// buffer, so the hardware returns 0 instead of reading; the caller masks the result.  Loads
// without branches around them keep the compiler's wait counts exact (a wait after a branch
// that may have issued a load has to assume it did, and vector loads complete in order).
struct Gather {
  __amdgpu_buffer_rsrc_t A_rowptr, P_rowptr, A_col, P_col, P_val, A_val, slot, pext;
  const double* A_val_ptr;  // the same values by address (read so where they pass 2 GiB)
};

// A value by 64-bit address, for arrays past the 2 GiB that a buffer offset reaches.  An invalid
// entry (idx < 0) reads entry 0 and returns 0, so the load is still issued unconditionally.
__device__ __forceinline__ double ld_dbl_wide(const double* __restrict__ p, int idx) {
  const double v = p[idx < 0 ? 0 : idx];
  return idx < 0 ? 0.0 : v;
}

template <bool PEXT>
__device__ __forceinline__ Stage3 st_entries(const Stage2& q, const Gather& g, int sub) {
  Stage3 r{q.I, -1, -1, -1, -1};
  r.t = q.I >= 0 && q.a0 + sub < q.a1 ? q.a0 + sub : -1;
  r.e = q.I >= 0 && q.p0 + sub < q.p1 ? q.p0 + sub : -1;
  r.J = ld_i32(PEXT ? g.pext : g.A_col, r.t);
  r.pi = ld_i32(g.P_col, r.e);
  return r;
}
template <bool PEXT, bool WIDE>
__device__ __forceinline__ Stage4 st_pext(const Stage3& q, const Gather& g) {
  Stage4 r{q.I, 0, 0, q.t, q.pi, q.e, -1, 0.0, 0.0};
  if (PEXT) {
    r.ps = (int)((unsigned)q.J >> 6);  // 0 for no entry (the load returned 0); unsigned: the
                                        // start may use the sign bit
    r.pe = r.ps + (q.J & 63);
  } else {
    const v2u pr = ld_pair(g.P_rowptr, q.t >= 0 ? q.J : -1);
    r.ps = (int)pr[0];
    r.pe = (int)pr[1];
  }
  r.av = WIDE ? ld_dbl_wide(g.A_val_ptr, q.t) : ld_dbl(g.A_val, q.t);
  const int sl = ld_i32(g.slot, q.e >= 0 ? q.pi : -1);
  r.sl = q.e >= 0 ? sl : -1;
  r.pw = ld_dbl(g.P_val, q.e);
  return r;
}

// One tile of the owner fold by the whole workgroup (NW wavefronts); smem holds the tile and the
// per-wavefront hash tables.  Ends with the tile written to C and a workgroup barrier.
// LONGC: the tile has rows of C longer than 2 * kHalf columns (R_I has at most 32 keys); an
// owned entry whose row of C is that long is folded key by key (see the fold).
template <int NW, bool PEXT, bool WIDE, bool LONGC>
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

  const int step = 2 * NW;
  const int nnzP = p.P_rowptr[p.n];
  const __amdgpu_buffer_rsrc_t rA = buffer_rsrc(p.A_rowptr, (unsigned)(p.n + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rP = buffer_rsrc(p.P_rowptr, (unsigned)(p.n + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rPc = buffer_rsrc(p.P_col, (unsigned)nnzP * 4u);
  const __amdgpu_buffer_rsrc_t rPv = buffer_rsrc(a.P_val, (unsigned)nnzP * 8u);
  const unsigned nnzA = (unsigned)p.A_rowptr[p.n];
  const __amdgpu_buffer_rsrc_t rAv = buffer_rsrc(a.A_val, WIDE ? 0u : nnzA * 8u);
  const Gather g{rA, rP, buffer_rsrc(p.A_col, nnzA * 4u), rPc, rPv, rAv,
                 buffer_rsrc(ts.slot, (unsigned)p.m * 4u), buffer_rsrc(a.A_pext, PEXT ? nnzA * 4u : 0u),
                 a.A_val};
  const unsigned hmul = a.hash_mul;
  const int npass = a.part < 0 ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int part = a.part < 0 ? (pass == 0 ? PART_OFF : PART_ON) : a.part;
    // the first of two passes walks only the tile's rows with off-block entries (Alg. 8, loop 1)
    const bool off_list = pass == 0 && npass == 2 && a.off_fptr != nullptr;
    const int* fine = off_list ? a.off_fine : tile_fine;
    const int f0 = off_list ? a.off_fptr[tile] : tile_fptr[tile];
    const int f1 = off_list ? a.off_fptr[tile + 1] : tile_fptr[tile + 1];
    // Software pipeline over the wavefront's row pairs f, f+step, f+2*step, ...: while the
    // pair being folded (cur) works in LDS, the next two pairs advance one load stage each
    // (entries of A and P -> extent of the row of P), so each dependent load overlaps one
    // iteration of LDS work instead of stalling the wavefront.  Row headers come from a block
    // loaded once per 32 iterations.
    const int fb = f0 + 2 * wid + half;
    int it0 = 0;
    Stage2 hb = hdr_load(fine, fb + sub * step, f1, rA, rP);
    Stage4 cur = st_pext<PEXT, WIDE>(st_entries<PEXT>(hdr_get(hb, 0, half), g, sub), g);
    Stage3 nxt = st_entries<PEXT>(hdr_get(hb, 1, half), g, sub);
    for (int it = 0, f = f0 + 2 * wid; f < f1; ++it, f += step) {
      // (1) owned entries of P(I,:) of cur: the ones whose column is a row of this tile
      const bool in_t = cur.sl >= 0 && (cur.sl >> kTileRowBits) == tile &&
                        part_takes(part, cur.I, cur.pi, p.n, p.m, a.K);
      const unsigned long long own = ballot(in_t);
      const unsigned own0 = (unsigned)own, own1 = (unsigned)(own >> 32);
      // (2) the products of cur's row, 32 per step: lane q's A entry owns products
      // [incl - len, incl) of the row; a nonempty segment of rank r leaves its weight and its
      // offset into P in rec[r]; product k belongs to the segment of rank #{ends <= k}
      const int len = cur.pe - cur.ps;
      const int incl = half_incl_scan(len);
      const int T0 = own0 ? __builtin_amdgcn_readlane(incl, 31) : 0;
      const int T1 = own1 ? __builtin_amdgcn_readlane(incl, 63) : 0;
      const int Th = half ? T1 : T0;
      const unsigned long long nonempty = ballot(len > 0);
      if (len > 0 && Th > 0) {
        const int r = prefix_count(nonempty) - (half ? __popc((unsigned)nonempty) : 0);
        hs->rec[half][r] = SegRec{cur.av, cur.ps - (incl - len), 0};
      }
      wave_sync();
      const int nstep = (max(T0, T1) + kHalf - 1) / kHalf;
      int before = 0;  // nonempty segments that end at or before the current window
      // the entries of P for the first kPrefetch steps (all of them for rows of up to 128
      // products) are requested together, so their latencies overlap; later steps one by one
      ProdLoad pq[kPrefetch];
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u)
        pq[u] = u < nstep ? prod_load(u, incl, len, Th, sub, half, before, hs->rec[half], rPc, rPv)
                          : ProdLoad{0, 0.0, 0.0, false};
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u)
        if (pq[u].ok) hash_add64(keys, vals, pq[u].j, pq[u].w * pq[u].v, hmul);
      for (int st = kPrefetch; st < nstep; ++st) {
        const ProdLoad cu = prod_load(st, incl, len, Th, sub, half, before, hs->rec[half], rPc, rPv);
        if (cu.ok) hash_add64(keys, vals, cu.j, cu.w * cu.v, hmul);
      }
      wave_sync();
      // (3) one load stage for each of the next two pairs.  Issued after the products' loads
      // have been consumed (a wait on a vector load also waits for all loads issued before it),
      // these fly during the fold, which works in LDS only.
      int k = it + 2 - it0;
      if (k == kHalf) {
        it0 += kHalf;
        k = 0;
        hb = hdr_load(fine, fb + (it0 + sub) * step, f1, rA, rP);
      }
      const Stage2 h2 = hdr_get(hb, k, half);
      const Stage4 nxt4 = st_pext<PEXT, WIDE>(nxt, g);
      const Stage3 nn3 = st_entries<PEXT>(h2, g, sub);
      // (4) fold the owned part of P(I,:) (x) R_I into the tile, one owned entry per half at a
      // time.  The owned entries leave (row start, row end, weight) in the half's records (free
      // once the products are in), compacted by rank, and every lane reads them back with one
      // broadcast LDS read per entry.
      {
        const unsigned hm = half ? own1 : own0;
        if (in_t) {
          const int rl = cur.sl & (kTileRows - 1);
          const int pos = __popc(hm & ((1u << sub) - 1u));
          hs->rec[half][pos] = SegRec{cur.pw, trp[rl], trp[rl + 1]};
        }
        wave_sync();
        const int nsel = __popc(hm);
        const int nmax = max(__popc(own0), __popc(own1));
        for (int kk = 0; kk < nmax; ++kk) {
          const SegRec rc = hs->rec[half][kk];
          const int c0 = kk < nsel ? rc.base : 0, c1 = kk < nsel ? rc.pad : 0;
          if (LONGC && c1 - c0 > 2 * kHalf) {
            // A row of C much longer than R_I: walking it would look up mostly columns that R_I
            // lacks.  Instead each lane takes the keys in its two slots of the table and finds
            // their positions in the row (its columns are sorted) by binary search; every key of
            // R_I is a column of C(i,:) (C's pattern is the structural product).
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
              const int sidx = sub + h2 * kHalf;
              const int j = keys[sidx];
              if (j != EMPTY) {
                int lo = c0, hi = c1;
                while (lo < hi) {
                  const int mid = (lo + hi) >> 1;
                  if (tc[mid] < j)
                    lo = mid + 1;
                  else
                    hi = mid;
                }
                if (lo < c1 && tc[lo] == j) atomicAdd(tv + lo, rc.w * vals[sidx]);
              }
            }
          } else {
            for (int c = c0 + sub; c < c1; c += kHalf) {
              const int j = tc[c];
              const int s = hash_find64(keys, j, hmul);
              if (s >= 0) atomicAdd(tv + c, rc.w * vals[s]);
            }
          }
        }
      }
      wave_sync();
      if (Th > 0) {
        keys[sub] = EMPTY;
        keys[sub + kHalf] = EMPTY;
        vals[sub] = 0.0;
        vals[sub + kHalf] = 0.0;
      }
      wave_sync();
      cur = nxt4;
      nxt = nn3;
    }
  }
  __syncthreads();
  tile_store(ts.rows, tp, nr, a.C_rowptr, trp, tv, a.C_val);
  __syncthreads();
}

template <int NW, bool PEXT, bool WIDE, bool LONGC>
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
  owner_fast_tile<NW, PEXT, WIDE, LONGC>(a, tiles[b], ts, tile_fptr, tile_fine, TE, smem);
}

// Batched form: a persistent grid works through a list of (plan, tile) items, every item one tile
// of one plan's owner fold.  The list (plan by plan, tiles in order) is cut into 8 contiguous
// chunks with a counter each; the workgroups of XCD x (workgroups are dispatched to the XCDs
// round-robin) take items from chunk x, so neighbouring tiles share that XCD's L2, and then help
// with the other chunks.  The batched form reads the row pointers of P (no numeric cache).
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
      owner_fast_tile<NW, false, false, false>(pl.a, tl, pl.ts, pl.tile_fptr, pl.tile_fine, pl.TE, smem);
    }
  }
}

size_t owner_fast_lds_bytes(int TE, int nw) {
  return (((size_t)TE * 12 + ((size_t)kTileRows + 1) * 4 + 15) / 16) * 16 + (size_t)nw * sizeof(HalfScratch);
}

template <bool PEXT, bool WIDE, bool LONGC>
static void launch_fast_nw(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                           const int* tile_fptr, const int* tile_fine, int TE, int nw, int remap,
                           size_t lds, hipStream_t s) {
  if (nw == 16)
    hipLaunchKernelGGL((k_owner_fast<16, PEXT, WIDE, LONGC>), dim3(tc.count), dim3(16 * WAVE), lds, s, a,
                       tc.tiles, ts, tile_fptr, tile_fine, TE, remap);
  else if (nw == 8)
    hipLaunchKernelGGL((k_owner_fast<8, PEXT, WIDE, LONGC>), dim3(tc.count), dim3(8 * WAVE), lds, s, a,
                       tc.tiles, ts, tile_fptr, tile_fine, TE, remap);
  else
    hipLaunchKernelGGL((k_owner_fast<4, PEXT, WIDE, LONGC>), dim3(tc.count), dim3(4 * WAVE), lds, s, a,
                       tc.tiles, ts, tile_fptr, tile_fine, TE, remap);
}

template <bool PEXT, bool WIDE>
static void launch_fast_longc(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                              const int* tile_fptr, const int* tile_fine, int TE, int nw, int remap,
                              size_t lds, hipStream_t s) {
  if (tc.long_c)
    launch_fast_nw<PEXT, WIDE, true>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
  else
    launch_fast_nw<PEXT, WIDE, false>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
}

hipError_t launch_owner_fast(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                             const int* tile_fptr, const int* tile_fine, int TE, int nw,
                             bool xcd_remap, hipStream_t s) {
  if (tc.count == 0) return hipSuccess;
  const size_t lds = owner_fast_lds_bytes(TE, nw);
  const int remap = xcd_remap ? 1 : 0;
  if (a.A_pext && a.wide_a)
    launch_fast_longc<true, true>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
  else if (a.A_pext)
    launch_fast_longc<true, false>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
  else if (a.wide_a)
    launch_fast_longc<false, true>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
  else
    launch_fast_longc<false, false>(a, tc, ts, tile_fptr, tile_fine, TE, nw, remap, lds, s);
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
