// Numeric merged product with the owner fold, staged-tile form, and the symbolic pass that lists
// each tile's halo.
//
// A workgroup owns a tile of rows of C (as in owner.hip) and first copies into LDS everything the
// tile's fine rows read from P: the rows P(J,:) of every J in the tile's halo (the columns of
// A(I,:) over the tile's fine rows I, and those rows I themselves).  Every product
// A(I,J) * P(J,j) then reads P from LDS instead of gathering it from memory.  Coarse columns are
// renumbered inside the tile (local ids 0 .. |U|-1 over the columns of the staged rows), and a
// table M[q][u] gives the position of local column u in the tile's q-th row of C.
//
// R_I is held in the positions of one row of C: for the tile's first row i0 among the columns of
// P(I,:), the columns of R_I are among those of C(i0,:) (C's pattern is the structural product,
// Eq. allatoncerow), so R_I(j) lives at the position of j in C(i0,:).  A wavefront takes 16 fine
// rows at a time, 4 lanes per row; the lanes of a row walk the entries A(I,J) in order and, for
// each, spread the entries of P(J,:) over the 4 lanes.  The columns of one row of P are distinct,
// so no two lanes of a row add into the same position of R_I in one instruction (an LDS atomic
// costs about 12 cycles more for every further lane on the same address), and the sixteen rows
// have their own R.  The fold C(i,:) += P(I,i) R_I for the owned columns i of P(I,:) (Eq.
// allatonceoutproduct restricted to the tile's rows) adds into the tile in LDS, which is written
// to C once at the end.
#include "device.hpp"
#include "internal.hpp"

namespace ptapk {

namespace {
constexpr unsigned kFib = 0x9E3779B1u;

// Insert key >= 0 into an LDS key table of 2^lg slots (linear probing, bounded by the table size).
// Returns false when no slot was found; *fresh tells whether this call stored the key.
__device__ __forceinline__ bool key_insert(int* keys, int lg, int key, bool* fresh) {
  const unsigned mask = (1u << lg) - 1u;
  unsigned s = ((unsigned)key * kFib) >> (32 - lg);
  for (int it = 0; it <= (int)mask; ++it) {
    const int k = keys[s];
    if (k == key) {
      *fresh = false;
      return true;
    }
    if (k == EMPTY) {
      const int old = atomicCAS(keys + s, EMPTY, key);
      if (old == EMPTY) {
        *fresh = true;
        return true;
      }
      if (old == key) {
        *fresh = false;
        return true;
      }
    }
    s = (s + 1) & mask;
  }
  *fresh = false;
  return false;
}

// Slot of key in a completed key table, or -1.
__device__ __forceinline__ int key_find(const int* keys, int lg, int key) {
  const unsigned mask = (1u << lg) - 1u;
  unsigned s = ((unsigned)key * kFib) >> (32 - lg);
  for (int it = 0; it <= (int)mask; ++it) {
    const int k = keys[s];
    if (k == key) return (int)s;
    if (k == EMPTY) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

// Exclusive prefix sum of a[0..L) in LDS by the whole workgroup; *total receives the sum.  wtot
// holds one int per wavefront.  Ends with a workgroup barrier.
__device__ void block_excl_scan(int* a, int L, int* wtot, int* total) {
  const int tid = threadIdx.x, nt = blockDim.x, wid = tid / WAVE;
  const int per = (L + nt - 1) / nt;
  const int b = min(L, tid * per), e = min(L, b + per);
  int sum = 0;
  for (int i = b; i < e; ++i) sum += a[i];
  const int incl = wave_incl_scan(sum);
  if (lane() == WAVE - 1) wtot[wid] = incl;
  __syncthreads();
  int run = incl - sum;
  for (int w = 0; w < wid; ++w) run += wtot[w];
  for (int i = b; i < e; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  if (tid == nt - 1) *total = run;
  __syncthreads();
}
}  // namespace

// =============================================================================================
// Symbolic: the halo of every tile (sorted fine rows whose rows of P the tile's fine rows read).
// Count pass (FILL = false), one workgroup per tile: stats[6t + 0..5] = number of halo rows,
// entries of P in them, distinct coarse columns among those entries, longest row of A and of P
// over the tile's fine rows, and 1 if a table overflowed.  Fill pass: the sorted halo rows of the
// listed tiles at halo_ptr[tile].
// =============================================================================================
constexpr int kHaloThreads = 256;
constexpr int kHaloKeysLog = 13;   // 8192 slots: at most kStagedMaxHalo halo rows
constexpr int kHaloUKeysLog = 12;  // 4096 slots: at most kStagedMaxCols coarse columns

template <bool FILL>
__global__ __launch_bounds__(kHaloThreads) void k_tile_halo(Patterns p, const int* __restrict__ tiles,
                                                            const int* __restrict__ tile_fptr,
                                                            const int* __restrict__ tile_fine,
                                                            int* __restrict__ stats,
                                                            const int* __restrict__ halo_ptr,
                                                            int* __restrict__ halo_rows) {
  __shared__ int keys[1 << kHaloKeysLog];
  __shared__ int ukeys[1 << kHaloUKeysLog];  // fill pass: the sort buffer
  __shared__ int cnt[4];                     // halo rows, entries of P, columns, overflow
  __shared__ int mx[2];
  const int t = tiles[blockIdx.x];
  const int tid = threadIdx.x, ln = lane(), wid = tid / WAVE, nw = kHaloThreads / WAVE;
  for (int i = tid; i < (1 << kHaloKeysLog); i += kHaloThreads) keys[i] = EMPTY;
  for (int i = tid; i < (1 << kHaloUKeysLog); i += kHaloThreads) ukeys[i] = EMPTY;
  if (tid < 4) cnt[tid] = 0;
  if (tid < 2) mx[tid] = 0;
  __syncthreads();
  const int f0 = tile_fptr[t], f1 = tile_fptr[t + 1];
  for (int f = f0 + wid; f < f1; f += nw) {
    const int I = tile_fine[f];
    const int a0 = p.A_rowptr[I], a1 = p.A_rowptr[I + 1];
    if (ln == 0) {
      atomicMax(&mx[0], a1 - a0);
      atomicMax(&mx[1], p.P_rowptr[I + 1] - p.P_rowptr[I]);
    }
    // k = a0 - 1 stands for the row I itself (its row of P gives the fold's weights)
    for (int k = a0 - 1 + ln; k < a1; k += WAVE) {
      const int J = k < a0 ? I : p.A_col[k];
      bool fresh;
      if (!key_insert(keys, kHaloKeysLog, J, &fresh)) {
        cnt[3] = 1;
        continue;
      }
      if (FILL || !fresh) continue;
      atomicAdd(&cnt[0], 1);
      const int ps = p.P_rowptr[J], pe = p.P_rowptr[J + 1];
      atomicAdd(&cnt[1], pe - ps);
      for (int e = ps; e < pe; ++e) {
        bool uf;
        if (!key_insert(ukeys, kHaloUKeysLog, p.P_col[e], &uf)) {
          cnt[3] = 1;
          break;
        }
        if (uf) atomicAdd(&cnt[2], 1);
      }
    }
  }
  __syncthreads();
  if (!FILL) {
    if (tid == 0) {
      int* o = stats + 6 * (size_t)t;
      o[0] = cnt[0];
      o[1] = cnt[1];
      o[2] = cnt[2];
      o[3] = mx[0];
      o[4] = mx[1];
      o[5] = cnt[3];
    }
    return;
  }
  // collect the keys (at most the sort buffer's size: the host fills only tiles that fit), sort
  // them ascending (bitonic network over the next power of two, padded with INT_MAX), write
  if (tid == 0) cnt[0] = 0;
  __syncthreads();
  constexpr int kBuf = 1 << kHaloUKeysLog;
  for (int s = tid; s < (1 << kHaloKeysLog); s += kHaloThreads) {
    const int k = keys[s];
    if (k != EMPTY) {
      const int pos = atomicAdd(&cnt[0], 1);
      if (pos < kBuf) ukeys[pos] = k;
    }
  }
  __syncthreads();
  const int nh = min(cnt[0], kBuf);
  int L = 1;
  while (L < nh) L <<= 1;
  for (int i = nh + tid; i < L; i += kHaloThreads) ukeys[i] = 0x7FFFFFFF;
  __syncthreads();
  for (int k = 2; k <= L; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < L; i += kHaloThreads) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = ukeys[i], y = ukeys[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            ukeys[i] = y;
            ukeys[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const int hp = halo_ptr[t];
  const int hn = halo_ptr[t + 1] - hp;
  for (int i = tid; i < min(nh, hn); i += kHaloThreads) halo_rows[hp + i] = ukeys[i];
}

hipError_t launch_tile_halo(const Patterns& p, const int* tiles, int ntiles, const int* tile_fptr,
                            const int* tile_fine, bool fill, int* stats, const int* halo_ptr,
                            int* halo_rows, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fill)
    hipLaunchKernelGGL(k_tile_halo<true>, dim3(ntiles), dim3(kHaloThreads), 0, s, p, tiles, tile_fptr,
                       tile_fine, stats, halo_ptr, halo_rows);
  else
    hipLaunchKernelGGL(k_tile_halo<false>, dim3(ntiles), dim3(kHaloThreads), 0, s, p, tiles, tile_fptr,
                       tile_fine, stats, halo_ptr, halo_rows);
  return hipGetLastError();
}

// =============================================================================================
// Numeric: the staged-tile kernel.
// =============================================================================================
namespace {
constexpr int kStG = 4;                  // lanes per fine row
constexpr int kStRows = WAVE / kStG;     // fine rows per wavefront
constexpr int kStSlots = kStagedMaxA / kStG;  // entries of A(I,:) per lane
constexpr int kStRStride = kStagedMaxRank + 1;  // doubles per R_I (padded against bank conflicts)

typedef unsigned v2u_t __attribute__((ext_vector_type(2)));
constexpr int kRawFlags = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawFlags);
}
// Loads through buffer resources: an index past the end (or -1) reads 0 instead of faulting.
__device__ __forceinline__ int bld_i32(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0);
}
__device__ __forceinline__ double bld_f64(__amdgpu_buffer_rsrc_t r, int idx) {
  const v2u_t v = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
__device__ __forceinline__ v2u_t bld_pair(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, idx * 4, 0, 0);
}

// Lane E of each group of four lanes, broadcast to the group (DPP quad permutation).  Every lane
// of the wavefront must be active.
template <int E>
__device__ __forceinline__ int qb(int v) {
  return __builtin_amdgcn_update_dpp(0, v, E * 0x55, 0xF, 0xF, false);
}
template <int E>
__device__ __forceinline__ double qbd(double v) {
  return __hiloint2double(qb<E>(__double2hiint(v)), qb<E>(__double2loint(v)));
}
__device__ __forceinline__ int quad_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));  // lanes [1,0,3,2]
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));  // lanes [2,3,0,1]
  return v;
}

// Halo-row table: key J, value (start of P(J,:) in the staged arrays) | (length << 24).
__device__ __forceinline__ int jh_find(const int2* jh, int lg, int J) {
  if (J < 0) return 0;
  const unsigned mask = (1u << lg) - 1u;
  unsigned s = ((unsigned)J * kFib) >> (32 - lg);
#pragma unroll 1
  for (int it = 0; it <= (int)mask; ++it) {
    const int2 kv = jh[s];
    if (kv.x == J) return kv.y;
    if (kv.x == EMPTY) return 0;
    s = (s + 1) & mask;
  }
  return 0;
}

struct StRow {  // one fine row at the A-entry stage (the same in the four lanes of its group)
  int I;        // fine row, or -1
  int J[kStSlots];
  double a[kStSlots];
};

}  // namespace

namespace {

// Up to kStagedMaxHalo / (kStagedWaves * 64) halo rows per thread in the set-up loops, all loads
// issued before any is used.
constexpr int kStHaloPer = kStagedMaxHalo / (kStagedWaves * WAVE);
constexpr int kStRowsPer = (kStagedMaxRows + kStagedWaves * WAVE - 1) / (kStagedWaves * WAVE);

// Four product steps of one batch: entry position `sub * 4 + e` of the rows P(J,:) of the
// entries A(I,J) at positions 4kk .. 4kk+3 of the row (broadcast from the group's lanes).
struct StBatch {
  int at[4];     // staged entry (0 where the step has no product)
  bool ok[4];    // the step has a product
  double a[4];   // A(I,J)
  int u[4];      // local column
  double v[4];   // P(J,j)
  int r[4];      // position of the column in the row's rank row
};

template <int KK, int SUB>
__device__ __forceinline__ void st_prep(const int (&sj)[kStSlots], const double (&av)[kStSlots], int e,
                                        StBatch& B) {
  const int s[4] = {qb<0>(sj[KK]), qb<1>(sj[KK]), qb<2>(sj[KK]), qb<3>(sj[KK])};
  B.a[0] = qbd<0>(av[KK]);
  B.a[1] = qbd<1>(av[KK]);
  B.a[2] = qbd<2>(av[KK]);
  B.a[3] = qbd<3>(av[KK]);
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int len = (int)((unsigned)s[x] >> 24);
    const int idx = kStG * SUB + e;
    B.ok[x] = idx < len;
    B.at[x] = B.ok[x] ? (s[x] & 0xFFFFFF) + idx : 0;
  }
}
__device__ __forceinline__ void st_load(const double* sval, const unsigned short* scol, StBatch& B) {
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    B.u[x] = scol[B.at[x]];
    B.v[x] = sval[B.at[x]];
  }
}
__device__ __forceinline__ void st_rank(const unsigned char* Mrow, StBatch& B) {
#pragma unroll
  for (int x = 0; x < 4; ++x) B.r[x] = Mrow[B.u[x]];
}
__device__ __forceinline__ void st_add(double* Rrow, const StBatch& B) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
    if (B.ok[x] && B.r[x] < kStagedMaxRank) atomicAdd(Rrow + B.r[x], B.a[x] * B.v[x]);
}

// Sub-steps 0 and 1 (entries 0..7 of the rows of P) of batch KK, with the loads of the next batch
// issued before this batch's adds.
template <int KK>
__device__ __forceinline__ void st_pipe(const int (&sj)[kStSlots], const double (&av)[kStSlots], int e,
                                        const double* sval, const unsigned short* scol,
                                        const unsigned char* Mrow, double* Rrow, StBatch (&B)[2]) {
  // B[0], B[1]: sub-steps 0 and 1 of batch KK, loads and ranks done
  StBatch N[2];
  if constexpr (KK + 1 < kStSlots) {
    st_prep<KK + 1, 0>(sj, av, e, N[0]);
    st_prep<KK + 1, 1>(sj, av, e, N[1]);
    st_load(sval, scol, N[0]);
    st_load(sval, scol, N[1]);
  }
  st_add(Rrow, B[0]);
  st_add(Rrow, B[1]);
  if constexpr (KK + 1 < kStSlots) {
    st_rank(Mrow, N[0]);
    st_rank(Mrow, N[1]);
    B[0] = N[0];
    B[1] = N[1];
  }
}

}  // namespace

template <int NW>
__global__ __launch_bounds__(NW * WAVE, 1) void k_staged(NumericArgs a, const int* __restrict__ tiles,
                                                        TileSet ts, const int* __restrict__ tile_fptr,
                                                        const int* __restrict__ tile_fine,
                                                        const int* __restrict__ halo_ptr,
                                                        const int* __restrict__ halo_rows,
                                                        StagedLayout L, int xcd_remap) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wtot[NW];
  __shared__ int scal[4];  // staged entries, local columns, tile entries
  static_assert(NW * WAVE * kStHaloPer >= kStagedMaxHalo, "halo rows per thread");
  const Patterns& p = a.p;
  int b = blockIdx.x;
  if (xcd_remap) {
    const int T = gridDim.x, q = T / 8, rem = T % 8, x = b % 8, k = b / 8;
    b = x * q + min(x, rem) + k;
  }
  const int tile = tiles[b];
  const int tid = threadIdx.x, nt = NW * WAVE, wid = tid / WAVE, ln = lane();

  double* sval = reinterpret_cast<double*>(smem + L.o_sval);
  double* tv = reinterpret_cast<double*>(smem + L.o_tv);
  double* R = reinterpret_cast<double*>(smem + L.o_R);
  int2* jh = reinterpret_cast<int2*>(smem + L.o_jh);
  unsigned short* scol = reinterpret_cast<unsigned short*>(smem + L.o_scol);
  unsigned short* tcl = reinterpret_cast<unsigned short*>(smem + L.o_tcl);
  int* trp = reinterpret_cast<int*>(smem + L.o_trp);
  unsigned short* own = reinterpret_cast<unsigned short*>(smem + L.o_own);
  unsigned char* M = smem + L.o_M;
  const int JH = 1 << L.JHlog, UH = 1 << L.UHlog;
  // set-up temporaries (in the R region)
  int* ukey = reinterpret_cast<int*>(smem + L.o_R);
  int* uid = ukey + UH;
  int* hJ = uid + UH;
  int* hps = hJ + L.NH;
  int* hst = hps + L.NH;       // NH + 1
  int* tcol = hst + L.NH + 1;  // SE
  int* tri = tcol + L.SE;      // NR: owned row index i
  unsigned short* tq = reinterpret_cast<unsigned short*>(tri + L.NR);  // TE: owned row of an entry
  int* tcs = reinterpret_cast<int*>(smem + L.o_tcs);  // start of C(i,:) of every owned row

  const int hp = halo_ptr[tile], nh = halo_ptr[tile + 1] - hp;
  const int tp = ts.ptr[tile], nr = ts.ptr[tile + 1] - tp;
  const int f0 = tile_fptr[tile], nf = tile_fptr[tile + 1] - f0;

  // (1) clear the tables; halo rows and the extents of their rows of P; owned rows of C and their
  // extents (every thread issues all of its loads before using any)
  for (int i = tid; i < JH; i += nt) jh[i] = make_int2(EMPTY, 0);
  for (int i = tid; i < UH; i += nt) ukey[i] = EMPTY;
  for (int i = tid; i < L.ULp; i += nt) own[i] = 0xFFFF;
  {
    unsigned* Mw = reinterpret_cast<unsigned*>(M);
    const int words = (L.NR * L.ULp) / 4;
    for (int i = tid; i < words; i += nt) Mw[i] = 0xFFFFFFFFu;
  }
  {
    int J[kStHaloPer];
#pragma unroll
    for (int u = 0; u < kStHaloPer; ++u) {
      const int h = tid + u * nt;
      J[u] = h < nh ? halo_rows[hp + h] : 0;
    }
#pragma unroll
    for (int u = 0; u < kStHaloPer; ++u) {
      const int h = tid + u * nt;
      if (h < nh) {
        const int ps = p.P_rowptr[J[u]], pe = p.P_rowptr[J[u] + 1];
        hJ[h] = J[u];
        hps[h] = ps;
        hst[h] = pe - ps;
      }
    }
    int I[kStRowsPer];
#pragma unroll
    for (int u = 0; u < kStRowsPer; ++u) {
      const int q = tid + u * nt;
      I[u] = q < nr ? ts.rows[tp + q] : 0;
    }
#pragma unroll
    for (int u = 0; u < kStRowsPer; ++u) {
      const int q = tid + u * nt;
      if (q < nr) {
        const int cs = a.C_rowptr[I[u]], ce = a.C_rowptr[I[u] + 1];
        tri[q] = I[u];
        tcs[q] = cs;
        trp[q] = ce - cs;
      }
    }
  }
  __syncthreads();
  // (2) starts of the staged rows and of the tile's rows
  block_excl_scan(hst, nh, wtot, &scal[0]);
  block_excl_scan(trp, nr, wtot, &scal[2]);
  if (tid == 0) {
    hst[nh] = scal[0];
    trp[nr] = scal[2];
  }
  __syncthreads();
  // (3) halo-row table; stage the values of P, collect its columns
#pragma unroll
  for (int u = 0; u < kStHaloPer; ++u) {
    const int h = tid + u * nt;
    if (h < nh) {
      const int J = hJ[h], ps = hps[h], st = hst[h], len = hst[h + 1] - st;
      const unsigned mask = (unsigned)JH - 1u;
      unsigned s = ((unsigned)J * kFib) >> (32 - L.JHlog);
      for (int it = 0; it < JH; ++it) {  // distinct keys: the first empty slot claimed is J's
        if (atomicCAS(&jh[s].x, EMPTY, J) == EMPTY) {
          jh[s].y = st | (len << 24);
          break;
        }
        s = (s + 1) & mask;
      }
      for (int e0 = 0; e0 < len; e0 += 4) {
        double v[4];
        int c[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int k = e0 + x < len ? ps + e0 + x : ps;
          v[x] = a.P_val[k];
          c[x] = p.P_col[k];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
          if (e0 + x < len) {
            sval[st + e0 + x] = v[x];
            tcol[st + e0 + x] = c[x];
            bool fresh;
            key_insert(ukey, L.UHlog, c[x], &fresh);
          }
      }
    }
  }
  __syncthreads();
  // (4) local column ids: the occupied slots of the column table in slot order
  for (int i = tid; i < UH; i += nt) uid[i] = ukey[i] != EMPTY ? 1 : 0;
  __syncthreads();
  block_excl_scan(uid, UH, wtot, &scal[1]);
  // (5) staged columns as local ids; owned row of every local column that is a row of the tile;
  // the tile's entries: owned row, local column, zero value
  const int S = scal[0], TEt = scal[2];
  for (int i = tid; i < S; i += nt) {
    const int sl = key_find(ukey, L.UHlog, tcol[i]);
    scol[i] = (unsigned short)(sl >= 0 ? uid[sl] : 0);
  }
  for (int q = tid; q < nr; q += nt) {
    const int sl = key_find(ukey, L.UHlog, tri[q]);
    if (sl >= 0) own[uid[sl]] = (unsigned short)q;
  }
  for (int c0 = 0; c0 < TEt; c0 += 4 * nt) {
    int col[4], qq[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int c = c0 + x * nt + tid;
      // owned row of entry c: the last q with trp[q] <= c
      int lo = 0, hi = nr;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (trp[mid] <= c) lo = mid; else hi = mid;
      }
      qq[x] = lo;
      col[x] = c < TEt ? a.C_col[tcs[lo] + (c - trp[lo])] : 0;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int c = c0 + x * nt + tid;
      if (c < TEt) {
        const int sl = key_find(ukey, L.UHlog, col[x]);
        tcl[c] = (unsigned short)(sl >= 0 ? uid[sl] : 0xFFFF);
        tq[c] = (unsigned short)qq[x];
        tv[c] = 0.0;
      }
    }
  }
  __syncthreads();
  // (6) position table M; R cleared (the temporaries are no longer needed after this)
  for (int c = tid; c < TEt; c += nt) {
    const int u = tcl[c], q = tq[c];
    if (u < L.ULp) M[(size_t)q * L.ULp + u] = (unsigned char)(c - trp[q]);
  }
  __syncthreads();
  for (int i = tid; i < NW * kStRows * kStRStride; i += nt) R[i] = 0.0;
  __syncthreads();

  // ---------------------------------------------------------------------------------------
  // Fine rows, 16 per wavefront and iteration (group g = lane / 4, e = lane % 4).
  // ---------------------------------------------------------------------------------------
  const int g = ln / kStG, e = ln % kStG;
  const unsigned nnzA = (unsigned)p.A_rowptr[p.n];
  const __amdgpu_buffer_rsrc_t rAc = rsrc(p.A_col, nnzA * 4u);
  const __amdgpu_buffer_rsrc_t rAv = rsrc(a.A_val, nnzA * 8u);
  const __amdgpu_buffer_rsrc_t rAp = rsrc(p.A_rowptr, (unsigned)(p.n + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rFn = rsrc(tile_fine + f0, (unsigned)nf * 4u);
  double* Rw = R + (size_t)wid * kStRows * kStRStride;
  double* Rrow = Rw + g * kStRStride;
  const int step = NW * kStRows;

  // software pipeline: the fine row three iterations ahead, its row pointers two ahead, the
  // entries of A one ahead, all issued right after the current rows' table lookups so that they
  // have a whole iteration to arrive
  auto hdr = [&](int f) {
    const int v = bld_i32(rFn, f < nf ? f : -1);
    return f < nf ? v : -1;
  };
  auto entries = [&](int I, v2u_t rp, StRow& o) {
    o.I = I;
    const int a0 = (int)rp[0], alen = I >= 0 ? (int)rp[1] - a0 : 0;
#pragma unroll
    for (int kk = 0; kk < kStSlots; ++kk) {
      const int k = e + kStG * kk;
      const int idx = k < alen ? a0 + k : -1;
      const int jv = bld_i32(rAc, idx);
      o.J[kk] = k < alen ? jv : -1;
      o.a[kk] = bld_f64(rAv, idx);
    }
  };
  int base = wid * kStRows;
  StRow cur;
  {
    const int I0 = hdr(base + g);
    entries(I0, bld_pair(rAp, I0), cur);
  }
  int I1 = hdr(base + step + g);
  v2u_t rp1 = bld_pair(rAp, I1);
  int I2 = hdr(base + 2 * step + g);
  for (; base < nf; base += step) {
    // halo lookups of the current rows' entries of A and of the rows themselves: first probes
    // together, further probes (rare) one by one
    int sj[kStSlots];
    int sI;
    {
      int2 kv[kStSlots + 1];
#pragma unroll
      for (int kk = 0; kk <= kStSlots; ++kk) {
        const int J = kk < kStSlots ? cur.J[kk] : cur.I;
        kv[kk] = jh[((unsigned)(J < 0 ? 0 : J) * kFib) >> (32 - L.JHlog)];
      }
      unsigned miss = 0;
#pragma unroll
      for (int kk = 0; kk <= kStSlots; ++kk) {
        const int J = kk < kStSlots ? cur.J[kk] : cur.I;
        const int val = J >= 0 && kv[kk].x == J ? kv[kk].y : 0;
        if (J >= 0 && kv[kk].x != J && kv[kk].x != EMPTY) miss |= 1u << kk;
        if (kk < kStSlots) sj[kk] = val; else sI = val;
      }
      if (miss) {
#pragma unroll
        for (int kk = 0; kk <= kStSlots; ++kk)
          if (miss & (1u << kk)) {
            const int v = jh_find(jh, L.JHlog, kk < kStSlots ? cur.J[kk] : cur.I);
            if (kk < kStSlots) sj[kk] = v; else sI = v;
          }
      }
    }
    StRow nx;
    entries(I1, rp1, nx);
    const v2u_t rp2 = bld_pair(rAp, I2);
    const int I3 = hdr(base + 3 * step + g);
    // owned entries of P(I,:) (positions e and e + 4): weight, owned row, start of its tile row
    const int lenI = (int)((unsigned)sI >> 24), stI = sI & 0xFFFFFF;
    int q0o = -1, q1o = -1;
    double w0 = 0.0, w1 = 0.0;
    {
      const int at0 = e < lenI ? stI + e : 0, at1 = e + kStG < lenI ? stI + e + kStG : 0;
      const int u0 = scol[at0], u1 = scol[at1];
      const double v0 = sval[at0], v1 = sval[at1];
      const int o0 = own[u0], o1 = own[u1];
      if (e < lenI && o0 != 0xFFFF) {
        q0o = o0;
        w0 = v0;
      }
      if (e + kStG < lenI && o1 != 0xFFFF) {
        q1o = o1;
        w1 = v1;
      }
    }
    // the row's rank row: its first owned entry (smallest position)
    int key = 0x7FFFFFFF;
    if (q1o >= 0) key = ((e + kStG) << 16) | q1o;
    if (q0o >= 0) key = (e << 16) | q0o;
    key = quad_min(key);
    const int qz = key == 0x7FFFFFFF ? 0 : (key & 0xFFFF);
    const unsigned char* Mrow = M + (size_t)qz * L.ULp;
    const int zb = trp[qz], zl = trp[qz + 1] - zb;
    const int tq0 = trp[q0o < 0 ? 0 : q0o], tq1 = trp[q1o < 0 ? 0 : q1o];

    // products A(I,J) * P(J,j) into R_I: batches of the entries 4kk..4kk+3 of A(I,:), entries 0..7
    // of their rows of P (sub-steps 0 and 1), the next batch's loads issued before the adds
    {
      StBatch B[2];
      st_prep<0, 0>(sj, cur.a, e, B[0]);
      st_prep<0, 1>(sj, cur.a, e, B[1]);
      st_load(sval, scol, B[0]);
      st_load(sval, scol, B[1]);
      st_rank(Mrow, B[0]);
      st_rank(Mrow, B[1]);
      st_pipe<0>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<1>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<2>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<3>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<4>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<5>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      st_pipe<6>(sj, cur.a, e, sval, scol, Mrow, Rrow, B);
      // rows of P longer than eight entries: the remaining entries, batch by batch
      int lm = 0;
#pragma unroll
      for (int kk = 0; kk < kStSlots; ++kk) lm = max(lm, (int)((unsigned)sj[kk] >> 24));
      if (ballot(lm > 2 * kStG)) {
#pragma unroll
        for (int kk = 0; kk < kStSlots; ++kk) {
          const int s[4] = {qb<0>(sj[kk]), qb<1>(sj[kk]), qb<2>(sj[kk]), qb<3>(sj[kk])};
          const double aa[4] = {qbd<0>(cur.a[kk]), qbd<1>(cur.a[kk]), qbd<2>(cur.a[kk]), qbd<3>(cur.a[kk])};
          int l4 = 0;
#pragma unroll
          for (int x = 0; x < 4; ++x) l4 = max(l4, (int)((unsigned)s[x] >> 24));
          for (int sub = 2; ballot(kStG * sub < l4); ++sub) {
            StBatch X;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              const int len = (int)((unsigned)s[x] >> 24), idx = kStG * sub + e;
              X.ok[x] = idx < len;
              X.at[x] = X.ok[x] ? (s[x] & 0xFFFFFF) + idx : 0;
              X.a[x] = aa[x];
            }
            st_load(sval, scol, X);
            st_rank(Mrow, X);
            st_add(Rrow, X);
          }
        }
      }
    }
    wave_sync();
    // fold: every owned entry (q, w) of the sixteen rows adds w * R_I into row q of the tile.  The
    // entries are listed in LDS (owned row and group, start of the tile row, rank row of the
    // group, weight); the first half of the wavefront folds the first half of the list and the
    // second half the rest, one entry per half and instruction (lane r takes position r).
    {
      const unsigned long long b0 = ballot(q0o >= 0), b1 = ballot(q1o >= 0);
      const int n0 = __popcll(b0), nrec = n0 + __popcll(b1);
      int4* rec = reinterpret_cast<int4*>(smem + L.o_rec) + wid * 2 * WAVE;
      const int zpk = (zb << 16) | zl;  // zb < 65536 and zl <= kStagedMaxRank
      if (q0o >= 0) {
        const int k = prefix_count(b0);
        rec[k] = make_int4(q0o | (g << 16), tq0, __double2loint(w0), __double2hiint(w0));
      }
      if (q1o >= 0) {
        const int k = n0 + prefix_count(b1);
        rec[k] = make_int4(q1o | (g << 16), tq1, __double2loint(w1), __double2hiint(w1));
      }
      // the rank row of a record is its group's: kept beside the group's R
      if (e == 0) reinterpret_cast<int*>(Rrow)[2 * kStagedMaxRank] = zpk;
      wave_sync();
      const int half = ln / 32, r = ln % 32;
      const int nh = (nrec + 1) / 2;
      const int k0 = half ? nh : 0, k1 = half ? nrec : nh;
      for (int k = k0; k < k0 + nh; ++k) {
        if (k >= k1) break;
        const int4 x = rec[k];
        const int q = x.x & 0xFFFF, gg = x.x >> 16, tqb = x.y;
        const double w = __hiloint2double(x.w, x.z);
        const double* Rg = Rw + gg * kStRStride;
        const int z = reinterpret_cast<const int*>(Rg)[2 * kStagedMaxRank];
        const int zbb = z >> 16, zll = z & 0xFFFF;
        const bool on = r < zll;
        const int u = tcl[on ? zbb + r : 0];
        const double rv = Rg[r];
        const int pos = u < L.ULp ? M[(size_t)q * L.ULp + u] : 0xFF;
        if (on && pos != 0xFF) atomicAdd(tv + tqb + pos, w * rv);
      }
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < (kStRows * kStRStride + WAVE - 1) / WAVE; ++k) {
      const int i = k * WAVE + ln;
      if (i < kStRows * kStRStride) Rw[i] = 0.0;
    }
    wave_sync();
    cur = nx;
    I1 = I2;
    rp1 = rp2;
    I2 = I3;
  }
  __syncthreads();
  // write the tile: every owned row to its place in C (offsets kept in LDS)
  for (int q = wid; q < nr; q += NW) {
    const int o = trp[q], len = trp[q + 1] - o, cs = tcs[q];
    for (int k = ln; k < len; k += WAVE) a.C_val[cs + k] = tv[o + k];
  }
}

hipError_t launch_staged(const NumericArgs& a, const int* tiles, int ntiles, const TileSet& ts,
                         const int* tile_fptr, const int* tile_fine, const int* halo_ptr,
                         const int* halo_rows, const StagedLayout& L, bool xcd_remap, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_staged<kStagedWaves>, dim3(ntiles), dim3(kStagedWaves * WAVE), (size_t)L.total,
                     s, a, tiles, ts, tile_fptr, tile_fine, halo_ptr, halo_rows, L, xcd_remap ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ptapk
