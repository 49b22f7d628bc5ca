// Device-side building blocks shared by the kernels: wavefront scans and ballots, open-addressing
// hash tables (on-chip LDS or device memory), the flattened walk over the products
// A(I,J) * P(J,j) of one row of AP, and the contiguous block split of the 1D row partition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptapk {

constexpr int WAVE = 64;
constexpr int EMPTY = -1;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Orders LDS traffic of one wavefront: every lane's earlier LDS writes are visible to every
// lane's later LDS reads (LDS operations of a wavefront complete in issue order; the fences
// stop the compiler from moving accesses across this point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ int prefix_count(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int ln = lane();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    int t = __shfl_up(v, d, WAVE);
    if (ln >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, WAVE));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

// ------------------------------------------------------------------------------------------
// Open-addressing hash tables with linear probing.  Keys are int32 >= 0, EMPTY marks a free
// slot, capacity is a power of two and always larger than the number of distinct keys, so
// every probe sequence reaches either its key or a free slot.  Slot = Fibonacci hash of the key
// (top bits of key * 2^32/phi), which spreads the clustered column indices of a stencil row.
//   G = false: table in LDS (ds_* instructions);
//   G = true : table in device memory (spill for long rows).  Reads go to L2 (agent-scope
//              loads) because the table is updated with L2 atomics.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned hslot(int key, int shift) {
  return ((unsigned)key * 0x9E3779B1u) >> shift;
}

template <bool G>
__device__ __forceinline__ int ld_key(const int* p) {
  if constexpr (G)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}

template <bool G>
__device__ __forceinline__ double ld_val(const double* p) {
  if constexpr (G)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}

// Insert `key` (no-op if present).  Returns the slot; *fresh tells whether this call claimed it.
template <bool G>
__device__ __forceinline__ int hs_insert(int* keys, unsigned mask, int shift, int key, bool& fresh) {
  unsigned s = hslot(key, shift);
  while (true) {
    int k = ld_key<G>(keys + s);
    if (k == key) {
      fresh = false;
      return (int)s;
    }
    if (k == EMPTY) {
      int old = atomicCAS(keys + s, EMPTY, key);
      if (old == EMPTY) {
        fresh = true;
        return (int)s;
      }
      if (old == key) {
        fresh = false;
        return (int)s;
      }
    }
    s = (s + 1) & mask;
  }
}

// Slot of `key`, or -1 if absent.
template <bool G>
__device__ __forceinline__ int hs_find(const int* keys, unsigned mask, int shift, int key) {
  unsigned s = hslot(key, shift);
  while (true) {
    int k = ld_key<G>(keys + s);
    if (k == key) return (int)s;
    if (k == EMPTY) return -1;
    s = (s + 1) & mask;
  }
}

// R(key) += v (Alg. 3's "+=": insert the pair if absent, otherwise add).
template <bool G>
__device__ __forceinline__ void hm_add(int* keys, double* vals, unsigned mask, int shift, int key,
                                       double v) {
  bool fresh;
  int s = hs_insert<G>(keys, mask, shift, key, fresh);
  atomicAdd(vals + s, v);
}

// Reset a table of `cap` slots (keys to EMPTY, values to 0) by one wavefront.
template <bool G>
__device__ __forceinline__ void table_clear(int* keys, double* vals, int cap) {
  for (int s = lane(); s < cap; s += WAVE) {
    keys[s] = EMPTY;
    if (vals) vals[s] = 0.0;
  }
  if constexpr (G)
    __threadfence();
  else
    wave_sync();
}

__device__ __forceinline__ int log2_pow2(int cap) { return 31 - __clz(cap); }

// ------------------------------------------------------------------------------------------
// Flattened walk over the products of one row of AP (Alg. 1 / Alg. 3 loops):
//   for each J with A(I,J) stored (ascending), for each j with P(J,j) stored:
//       f(k, a) with k = position of P(J,j) in P's arrays and a = A(I,J).
// The (J, j) pairs are spread evenly over the 64 lanes: a wavefront prefix sum of the P-row
// lengths gives each A entry its range of product numbers q, and each lane finds the A entry
// that owns its q by binary lifting over those offsets (held in LDS).  Up to 64 A entries are
// handled per step, so rows of any length work.
// ------------------------------------------------------------------------------------------
struct WaveScratch {
  int off[WAVE];
  int ps[WAVE];
  double a[WAVE];
};

template <class F>
__device__ __forceinline__ void for_products(int a0, int a1, const int* __restrict__ A_col,
                                             const double* __restrict__ A_val,
                                             const int* __restrict__ P_rowptr, WaveScratch* ws,
                                             F&& f) {
  const int ln = lane();
  for (int base = a0; base < a1; base += WAVE) {
    const int t = base + ln;
    int ps = 0, pl = 0;
    double a = 0.0;
    if (t < a1) {
      const int J = A_col[t];
      ps = P_rowptr[J];
      pl = P_rowptr[J + 1] - ps;
      if (A_val) a = A_val[t];
    }
    const int incl = wave_incl_scan(pl);
    const int total = __shfl(incl, WAVE - 1, WAVE);
    ws->off[ln] = incl - pl;
    ws->ps[ln] = ps;
    ws->a[ln] = a;
    wave_sync();
    for (int q = ln; q < total; q += WAVE) {
      int lo = 0;
#pragma unroll
      for (int step = WAVE / 2; step > 0; step >>= 1)
        if (ws->off[lo + step] <= q) lo += step;
      f(ws->ps[lo] + (q - ws->off[lo]), ws->a[lo]);
    }
    wave_sync();
  }
}

// ------------------------------------------------------------------------------------------
// Owner tiles: a tile is a set of up to kTileRows rows of C, listed (ascending) in
// rows[ptr[t] .. ptr[t+1]).  slot[i] = t * kTileRows + (position of row i in its tile), so a
// single load tells whether column i of P belongs to the tile and where its row sits in LDS.
// ------------------------------------------------------------------------------------------
constexpr int kTileRowBits = 10;
constexpr int kTileRows = 1 << kTileRowBits;

struct TileSet {
  const int* ptr;
  const int* rows;
  const int* slot;
};

// Copy a tile's rows of C into LDS: trp[q] = offset of local row q (trp[nr] = entries), tc = the
// columns, tv = 0.  All threads of the workgroup take part; ends with a workgroup barrier.
__device__ __forceinline__ void tile_load(const int* __restrict__ rows, int tp, int nr,
                                          const int* __restrict__ C_rowptr,
                                          const int* __restrict__ C_col, int* trp, int* tc,
                                          double* tv) {
  const int wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE, ln = lane();
  if (wid == 0) {
    int run = 0;
    for (int q0 = 0; q0 < nr; q0 += WAVE) {
      const int q = q0 + ln;
      int len = 0;
      if (q < nr) {
        const int i = rows[tp + q];
        len = C_rowptr[i + 1] - C_rowptr[i];
      }
      const int incl = wave_incl_scan(len);
      if (q < nr) trp[q] = run + incl - len;
      run += __shfl(incl, WAVE - 1, WAVE);
    }
    if (ln == 0) trp[nr] = run;
  }
  __syncthreads();
  for (int q = wid; q < nr; q += nw) {
    const int i = rows[tp + q];
    const int s = C_rowptr[i], e = C_rowptr[i + 1], o = trp[q] - s;
    for (int k = s + ln; k < e; k += WAVE) {
      tc[o + k] = C_col[k];
      tv[o + k] = 0.0;
    }
  }
  __syncthreads();
}

// Write a tile's values back to the rows of C (each row contiguous in C).
__device__ __forceinline__ void tile_store(const int* __restrict__ rows, int tp, int nr,
                                           const int* __restrict__ C_rowptr, const int* trp,
                                           const double* tv, double* __restrict__ C_val) {
  const int wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE, ln = lane();
  for (int q = wid; q < nr; q += nw) {
    const int i = rows[tp + q];
    const int s = C_rowptr[i], e = C_rowptr[i + 1], o = trp[q] - s;
    for (int k = s + ln; k < e; k += WAVE) C_val[k] = tv[o + k];
  }
}

// Contiguous K-way split of [0, total) as in the 1D block-row partition (Section 2): block b
// owns [floor(b*total/K), floor((b+1)*total/K)).  The block of idx is the largest b with
// floor(b*total/K) <= idx, that is b*total <= (idx+1)*K - 1, so b = floor(((idx+1)*K - 1) / total).
// The quotient is below 2^31 and the FP64 product of num and the reciprocal of total carries a
// relative error of a few 2^-53, so its integer part is within one of b; the two 64-bit products
// (below 2^62) settle it.  Both 64-bit integer division and an IEEE FP64 division are long
// instruction sequences on the GPU, and this runs for every entry of P(I,:) in the two-pass
// forms; the reciprocal depends only on total, so the compiler takes it out of the loops (with
// a division in place the on-block test cost the all-at-once product 16% at 128^3, K = 8).
__device__ __forceinline__ int block_of(int idx, int total, int K) {
  if (K < (1 << 22) && (long long)total * K < (1LL << 31)) {
    // everything fits 32 bits: the FP32 estimate carries a relative error of at most 3 * 2^-24
    // and the quotient is below K < 2^22, so it is within one; 32-bit products settle it
    const int num32 = (idx + 1) * K - 1;
    int b = (int)((float)num32 * (1.0f / (float)total));
    while ((b + 1) * total <= num32) ++b;
    while (b > 0 && b * total > num32) --b;
    return b;
  }
  const long long num = (long long)(idx + 1) * K - 1;
  int b = (int)((double)num * (1.0 / (double)total));
  while ((long long)(b + 1) * total <= num) ++b;
  while (b > 0 && (long long)b * total > num) --b;
  return b;
}

// Which entries P(I,i) a pass folds: all of them (merged, Alg. 10), only the off-block ones
// (pass 1 of Alg. 8, P_o) or only the on-block ones (pass 2 of Alg. 8, P_d).
enum FoldPart { PART_ALL = 0, PART_OFF = 1, PART_ON = 2 };

__device__ __forceinline__ bool part_takes(int part, int I, int i, int n, int m, int K) {
  if (part == PART_ALL) return true;
  if (K <= 1) return part == PART_ON;  // one block: every entry is on-block
  const bool diag = block_of(I, n, K) == block_of(i, m, K);
  return part == PART_ON ? diag : !diag;
}

}  // namespace ptapk
