// HIP kernels for gfx950: input validation, pattern transpose, symbolic phase (row sizes of AP,
// pattern of C, owner tiles), the numeric all-at-once / merged folds (atomic and owner), the
// two-step comparison and the adjoint.
#include "device.hpp"
#include "host_logic.hpp"
#include "internal.hpp"

namespace ptapk {

namespace {

constexpr int kThreads = kWavesPerBlock * WAVE;

// Blocks for `count` items at `threads` per block, at most cap_blocks.  The default cap covers any
// int32 count with one thread per item at 256 threads per block (kernels without a grid-stride loop
// rely on it); launches over a grid-stride loop pass a smaller cap.
inline int grid_for(long long count, int threads, int cap_blocks = 1 << 23) {
  long long g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap_blocks) g = cap_blocks;
  return (int)g;
}

// Grid of a launch that gives one wavefront per row.  Spill launches (tables in device memory)
// use a fixed number of wavefronts that stride over the rows, so the workspace stays bounded.
inline int wave_grid(int count, bool global) {
  if (global) return kSpillWaves / kWavesPerBlock;
  return grid_for(count, kWavesPerBlock, 1 << 30);
}

// Device-memory table of wavefront `w` (global wave index) for spill launches.
__device__ __forceinline__ int* gkeys(int* gtab, int cap, int w) { return gtab + (size_t)w * cap; }

}  // namespace

// =============================================================================================
// Utilities
// =============================================================================================

template <class T>
__global__ void k_fill(T* p, T value, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

hipError_t launch_fill_i32(int* p, int value, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<int>, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

// Streaming read: every thread sums its 16-byte pairs in grid-stride order, then the wavefront
// and the workgroup reduce, and one device-wide add per workgroup goes into *out (zeroed first).
__global__ __launch_bounds__(256) void k_stream_sum(const double2* __restrict__ x, long long npairs,
                                                    const double* __restrict__ tail, int ntail,
                                                    double* out) {
  __shared__ double red[256 / WAVE];
  double acc = 0.0;
  for (long long k = blockIdx.x * 256LL + threadIdx.x; k < npairs; k += (long long)gridDim.x * 256) {
    const double2 v = x[k];
    acc += v.x + v.y;
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) acc += tail[threadIdx.x];
  acc = wave_sum(acc);
  if (lane() == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) t += red[w];
    atomicAdd(out, t);
  }
}

hipError_t launch_stream_sum(const double* x, long long n, double* out, hipStream_t s) {
  hipError_t e = launch_fill_f64(out, 0.0, 1, s);
  if (e != hipSuccess || n <= 0) return e;
  const long long npairs = n / 2;
  hipLaunchKernelGGL(k_stream_sum, dim3(grid_for(npairs, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x), npairs, x + 2 * npairs, (int)(n - 2 * npairs),
                     out);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double value, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, value,
                     count);
  return hipGetLastError();
}

__global__ void k_count_cols(const int* __restrict__ col, long long nnz, int* cnt) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nnz;
       k += (long long)gridDim.x * blockDim.x)
    atomicAdd(cnt + col[k], 1);
}

hipError_t launch_count_cols(const int* col, long long nnz, int* cnt, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, s, col, nnz, cnt);
  return hipGetLastError();
}

// Column index lists of a CSR pattern: for every stored (r, c), append r to list c and record
// the entry's position.  Order within a list follows the atomic cursor (not sorted).
__global__ void k_transpose_fill(const int* __restrict__ rowptr, const int* __restrict__ col,
                                 int nrows, int* cursor, int* t_row, int* t_pos) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    const int pos = atomicAdd(cursor + col[k], 1);
    t_row[pos] = r;
    if (t_pos) t_pos[pos] = k;
  }
}

hipError_t launch_transpose_fill(const int* rowptr, const int* col, int nrows, int* cursor,
                                 int* t_row, int* t_pos, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(nrows, 256)), dim3(256), 0, s, rowptr, col,
                     nrows, cursor, t_row, t_pos);
  return hipGetLastError();
}

// Fine-row statistics of a plan, reduced over all rows: out[0] counts the rows with P(I,:) and R_I
// both non-empty (the rows the fold needs), out[1] = sum_I nnz(P(I,:)) |R_I| (fold terms),
// out[2] = max_I |R_I|, out[3] = max_I max(nnz(P(I,:)), nnz(A(I,:))).  out holds zeros on entry.
// Launched with 256 threads per block, grid-stride over the rows.
__global__ void k_row_stats(Patterns p, const int* __restrict__ r, const int* __restrict__ w,
                            unsigned long long* out) {
  __shared__ unsigned long long sh[5][256];
  const int t = threadIdx.x;
  unsigned long long v[5] = {0, 0, 0, 0, 0};
  for (long long I = blockIdx.x * (long long)blockDim.x + t; I < p.n; I += (long long)gridDim.x * blockDim.x) {
    const int lp = p.P_rowptr[I + 1] - p.P_rowptr[I];
    const int la = p.A_rowptr[I + 1] - p.A_rowptr[I];
    const int rI = r[I];
    if (lp > 0 && rI > 0) {
      v[0] += 1;
      v[1] += (unsigned long long)lp * (unsigned long long)rI;
      v[4] += (unsigned long long)w[I];
    }
    v[2] = max(v[2], rI > 0 ? (unsigned long long)rI : 0ULL);
    const int l = lp > la ? lp : la;
    v[3] = max(v[3], l > 0 ? (unsigned long long)l : 0ULL);
  }
  for (int q = 0; q < 5; ++q) sh[q][t] = v[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      sh[0][t] += sh[0][t + h];
      sh[1][t] += sh[1][t + h];
      sh[2][t] = sh[2][t] > sh[2][t + h] ? sh[2][t] : sh[2][t + h];
      sh[3][t] = sh[3][t] > sh[3][t + h] ? sh[3][t] : sh[3][t + h];
      sh[4][t] += sh[4][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    atomicAdd(out + 4, sh[4][0]);
    atomicAdd(out, sh[0][0]);
    atomicAdd(out + 1, sh[1][0]);
    atomicMax(out + 2, sh[2][0]);
    atomicMax(out + 3, sh[3][0]);
  }
}

hipError_t launch_row_stats(const Patterns& p, const int* r, const int* w, unsigned long long* out,
                            hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  // grid-stride over at most 1024 workgroups: few same-address atomics at the end
  hipLaunchKernelGGL(k_row_stats, dim3(grid_for(p.n, 256, 1024)), dim3(256), 0, s, p, r, w, out);
  return hipGetLastError();
}

// =============================================================================================
// Sorted emission of a key set: compact the occupied slots of a table (ballot + prefix count)
// into `list`, then place every key at its rank (number of smaller keys) in `out`.
// =============================================================================================
template <bool G>
__device__ __forceinline__ int compact_keys(const int* keys, int cap, int* list) {
  const int ln = lane();
  int base = 0;
  for (int s0 = 0; s0 < cap; s0 += WAVE) {
    const int k = ld_key<G>(keys + s0 + ln);
    const unsigned long long mk = ballot(k != EMPTY);
    if (k != EMPTY) list[base + prefix_count(mk)] = k;
    base += __popcll(mk);
  }
  if constexpr (G)
    __threadfence();
  else
    wave_sync();
  return base;
}

template <bool G>
__device__ __forceinline__ void rank_sort_store(const int* list, int cnt, int* out) {
  for (int x = lane(); x < cnt; x += WAVE) {
    const int key = ld_key<G>(list + x);
    int rank = 0;
    for (int y = 0; y < cnt; ++y) rank += ld_key<G>(list + y) < key;
    out[rank] = key;
  }
}

// =============================================================================================
// Symbolic: |R_I| (Alg. 1 / Alg. 2: the size of the key set of row I of AP) and, for the
// two-step method, the sorted pattern of AP.
// =============================================================================================
template <bool G, bool FILL>
__global__ __launch_bounds__(kThreads) void k_ap_rows(Patterns p, const int* __restrict__ rows,
                                                      int count, int cap, int* r_out,
                                                      const int* __restrict__ AP_rowptr,
                                                      int* AP_col, int* gtab) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem) + wid;
  const int stride_t = cap + cap / 2;  // keys, then a list of up to cap/2 keys
  int* keys = G ? gkeys(gtab, stride_t, gw)
                : reinterpret_cast<int*>(smem + kWavesPerBlock * sizeof(WaveScratch)) + wid * stride_t;
  int* list = keys + cap;
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  table_clear<G>(keys, nullptr, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int I = rows[r];
    int fresh_cnt = 0;
    for_products(p.A_rowptr[I], p.A_rowptr[I + 1], p.A_col, nullptr, p.P_rowptr, ws,
                 [&](int k, double) {
                   bool fresh;
                   hs_insert<G>(keys, mask, shift, p.P_col[k], fresh);
                   fresh_cnt += fresh ? 1 : 0;
                 });
    if constexpr (FILL) {
      if constexpr (G) __threadfence();
      const int cnt = compact_keys<G>(keys, cap, list);
      rank_sort_store<G>(list, cnt, AP_col + AP_rowptr[I]);
    } else {
      fresh_cnt = wave_sum(fresh_cnt);
      if (ln == 0) r_out[I] = fresh_cnt;
    }
    table_clear<G>(keys, nullptr, cap);
  }
}

static size_t key_lds_bytes(int cap) {
  return kWavesPerBlock * (sizeof(WaveScratch) + (size_t)(cap + cap / 2) * sizeof(int));
}

hipError_t launch_ap_row_count(const Patterns& p, const RowClass& rc, int* r_out, int* gtab,
                               hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  if (rc.global)
    hipLaunchKernelGGL((k_ap_rows<true, false>), dim3(grid), dim3(kThreads),
                       kWavesPerBlock * sizeof(WaveScratch), s, p, rc.rows, rc.count, rc.cap, r_out,
                       nullptr, nullptr, gtab);
  else
    hipLaunchKernelGGL((k_ap_rows<false, false>), dim3(grid), dim3(kThreads), key_lds_bytes(rc.cap),
                       s, p, rc.rows, rc.count, rc.cap, r_out, nullptr, nullptr, gtab);
  return hipGetLastError();
}

hipError_t launch_ap_row_fill(const Patterns& p, const RowClass& rc, const int* AP_rowptr,
                              int* AP_col, int* gtab, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  if (rc.global)
    hipLaunchKernelGGL((k_ap_rows<true, true>), dim3(grid), dim3(kThreads),
                       kWavesPerBlock * sizeof(WaveScratch), s, p, rc.rows, rc.count, rc.cap,
                       nullptr, AP_rowptr, AP_col, gtab);
  else
    hipLaunchKernelGGL((k_ap_rows<false, true>), dim3(grid), dim3(kThreads), key_lds_bytes(rc.cap),
                       s, p, rc.rows, rc.count, rc.cap, nullptr, AP_rowptr, AP_col, gtab);
  return hipGetLastError();
}

// Upper bound on |C(i,:)|: C(i,:) is the union of S(R_I) over I with P(I,i) stored
// (Eq. allatoncerow), so |C(i,:)| <= min(m, sum of |R_I|).
__global__ void k_c_bound(const int* __restrict__ pt_ptr, const int* __restrict__ pt_row,
                          const int* __restrict__ r, int m, long long* bound) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  long long s = 0;
  for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) s += r[pt_row[t]];
  bound[i] = s < m ? s : m;
}

hipError_t launch_c_bound(const int* pt_ptr, const int* pt_row, const int* r, int m,
                          long long* bound, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_c_bound, dim3(grid_for(m, 256)), dim3(256), 0, s, pt_ptr, pt_row, r, m,
                     bound);
  return hipGetLastError();
}

// =============================================================================================
// Symbolic: pattern of C by rows (Eq. allatoncerow).  All-at-once / merged: S(C(i,:)) is the
// union over I in the column list of P for i of S(R_I), with S(R_I) formed again from A and P
// (no AP is stored).  Two-step: the union of the stored rows of AP (Alg. 5, P^T (AP)).
// Count mode writes |C(i,:)|; fill mode writes the sorted columns.
// =============================================================================================
template <bool G, bool FILL, bool TWOSTEP>
__global__ __launch_bounds__(kThreads) void k_c_rows(Patterns p, const int* __restrict__ pt_ptr,
                                                     const int* __restrict__ pt_row,
                                                     const int* __restrict__ AP_rowptr,
                                                     const int* __restrict__ AP_col,
                                                     const int* __restrict__ rows, int count,
                                                     int cap, int* cnt_out,
                                                     const int* __restrict__ C_rowptr, int* C_col,
                                                     int* gtab) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem) + wid;
  const int stride_t = cap + cap / 2;
  int* keys = G ? gkeys(gtab, stride_t, gw)
                : reinterpret_cast<int*>(smem + kWavesPerBlock * sizeof(WaveScratch)) + wid * stride_t;
  int* list = keys + cap;
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  table_clear<G>(keys, nullptr, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int i = rows[r];
    int fresh_cnt = 0;
    for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) {
      const int I = pt_row[t];
      if constexpr (TWOSTEP) {
        for (int e = AP_rowptr[I] + ln; e < AP_rowptr[I + 1]; e += WAVE) {
          bool fresh;
          hs_insert<G>(keys, mask, shift, AP_col[e], fresh);
          fresh_cnt += fresh ? 1 : 0;
        }
      } else {
        for_products(p.A_rowptr[I], p.A_rowptr[I + 1], p.A_col, nullptr, p.P_rowptr, ws,
                     [&](int k, double) {
                       bool fresh;
                       hs_insert<G>(keys, mask, shift, p.P_col[k], fresh);
                       fresh_cnt += fresh ? 1 : 0;
                     });
      }
    }
    if constexpr (FILL) {
      if constexpr (G) __threadfence();
      const int cnt = compact_keys<G>(keys, cap, list);
      rank_sort_store<G>(list, cnt, C_col + C_rowptr[i]);
    } else {
      fresh_cnt = wave_sum(fresh_cnt);
      if (ln == 0) cnt_out[i] = fresh_cnt;
    }
    table_clear<G>(keys, nullptr, cap);
  }
}

hipError_t launch_c_rows(const Patterns& p, const int* pt_ptr, const int* pt_row,
                         const int* AP_rowptr, const int* AP_col, const RowClass& rc, bool fill,
                         int* cnt_out, const int* C_rowptr, int* C_col, int* gtab, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  const size_t lds = rc.global ? kWavesPerBlock * sizeof(WaveScratch) : key_lds_bytes(rc.cap);
  const bool two = AP_rowptr != nullptr;
#define PTAP_LAUNCH_C(G, F, T)                                                                   \
  hipLaunchKernelGGL((k_c_rows<G, F, T>), dim3(grid), dim3(kThreads), lds, s, p, pt_ptr, pt_row, \
                     AP_rowptr, AP_col, rc.rows, rc.count, rc.cap, cnt_out, C_rowptr, C_col, gtab)
  if (rc.global) {
    if (fill) {
      if (two) PTAP_LAUNCH_C(true, true, true); else PTAP_LAUNCH_C(true, true, false);
    } else {
      if (two) PTAP_LAUNCH_C(true, false, true); else PTAP_LAUNCH_C(true, false, false);
    }
  } else {
    if (fill) {
      if (two) PTAP_LAUNCH_C(false, true, true); else PTAP_LAUNCH_C(false, true, false);
    } else {
      if (two) PTAP_LAUNCH_C(false, false, true); else PTAP_LAUNCH_C(false, false, false);
    }
  }
#undef PTAP_LAUNCH_C
  return hipGetLastError();
}

// =============================================================================================
// Owner tiles: for each tile (a set of rows of C), the sorted distinct fine rows I with P(I,i)
// stored for some i in the tile (from P's column lists), the largest |R_I| among them and the
// longest of their rows of A and P.  A bitmap over windows of the candidates' index span removes duplicates and emits the
// rows in ascending order.
// =============================================================================================
constexpr int kTileBlock = 256;
constexpr int kWindowBits = 262144;  // 32 KiB of LDS: one window covers a 128^3 tile's candidates

__device__ __forceinline__ int block_reduce_min(int v, int* red) {
  v = -wave_max(-v);
  if (lane() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  int r = red[0];
  for (int w = 1; w < kTileBlock / WAVE; ++w) r = min(r, red[w]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ int block_reduce_max(int v, int* red) {
  v = wave_max(v);
  if (lane() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  int r = red[0];
  for (int w = 1; w < kTileBlock / WAVE; ++w) r = max(r, red[w]);
  __syncthreads();
  return r;
}

// Exclusive scan over the block; returns this thread's offset and writes the total.
__device__ __forceinline__ int block_excl_scan(int v, int* red, int& total) {
  const int incl = wave_incl_scan(v);
  if (lane() == WAVE - 1) red[threadIdx.x / WAVE] = incl;
  __syncthreads();
  int before = 0, tot = 0;
  for (int w = 0; w < kTileBlock / WAVE; ++w) {
    if (w < (int)(threadIdx.x / WAVE)) before += red[w];
    tot += red[w];
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

template <bool FILL>
__global__ __launch_bounds__(kTileBlock) void k_tile_fine(const int* __restrict__ pt_ptr,
                                                          const int* __restrict__ pt_row,
                                                          TileSet ts, const int* __restrict__ r,
                                                          const int* __restrict__ A_rowptr,
                                                          const int* __restrict__ P_rowptr,
                                                          int* cnt_out, int* rmax_out,
                                                          const int* __restrict__ fptr,
                                                          int* fine, int part, int n, int m, int K) {
  __shared__ unsigned bits[kWindowBits / 32];
  __shared__ int red[kTileBlock / WAVE];
  const int tile = blockIdx.x;
  const int tp = ts.ptr[tile], nr = ts.ptr[tile + 1] - tp;
  const int ts_n = n, ts_m = m;
  // candidates: the column lists of P for every row of the tile (one thread per tile row)
  int lo = INT32_MAX, hi = -1, rmax = 0, lmax = 0;
  for (int q = threadIdx.x; q < nr; q += kTileBlock) {
    const int i = ts.rows[tp + q];
    for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) {
      const int I = pt_row[t];
      if (!part_takes(part, I, i, ts_n, ts_m, K)) continue;
      lo = min(lo, I);
      hi = max(hi, I);
      if (!FILL) {
        rmax = max(rmax, r[I]);
        lmax = max(lmax, max(A_rowptr[I + 1] - A_rowptr[I], P_rowptr[I + 1] - P_rowptr[I]));
      }
    }
  }
  lo = block_reduce_min(lo, red);
  hi = block_reduce_max(hi, red);
  if (!FILL) {
    rmax = block_reduce_max(rmax, red);
    lmax = block_reduce_max(lmax, red);
  }
  int emitted = 0;
  for (long long wb = lo; wb <= hi; wb += kWindowBits) {
    for (int w = threadIdx.x; w < kWindowBits / 32; w += kTileBlock) bits[w] = 0u;
    __syncthreads();
    for (int q = threadIdx.x; q < nr; q += kTileBlock) {
      const int i = ts.rows[tp + q];
      for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) {
        if (!part_takes(part, pt_row[t], i, ts_n, ts_m, K)) continue;
        const long long d = (long long)pt_row[t] - wb;
        if (d >= 0 && d < kWindowBits) atomicOr(bits + (d >> 5), 1u << (d & 31));
      }
    }
    __syncthreads();
    constexpr int kWordsPerThread = kWindowBits / 32 / kTileBlock;
    int mine = 0;
    for (int q = 0; q < kWordsPerThread; ++q) mine += __popc(bits[threadIdx.x * kWordsPerThread + q]);
    int total;
    int pos = block_excl_scan(mine, red, total);
    if (FILL) {
      int* out = fine + fptr[tile] + emitted;
      for (int q = 0; q < kWordsPerThread; ++q) {
        const int wi = threadIdx.x * kWordsPerThread + q;
        unsigned bw = bits[wi];
        while (bw) {
          const int bit = __ffs(bw) - 1;
          bw &= bw - 1;
          out[pos++] = (int)(wb + wi * 32 + bit);
        }
      }
    }
    emitted += total;
    __syncthreads();
  }
  if (!FILL && threadIdx.x == 0) {
    cnt_out[tile] = emitted;
    rmax_out[2 * tile] = rmax;
    rmax_out[2 * tile + 1] = lmax;
  }
}

// Order each tile's fine-row list by the number of the row's entries of P that the tile owns
// (ascending, rows of equal count in ascending index order): the short-row owner kernel pairs
// consecutive rows in a wavefront and its fold takes as many steps as the larger of the two
// counts.  One workgroup per tile, a stable counting sort in LDS; lists longer than kOrderMax
// keep their ascending order.  The order costs cache locality (rows of P are fetched again
// between the sweeps of the count classes), so a tile with few distinct counts is ordered within
// windows of kTileBlock consecutive rows, which pairs as well there; a tile with many (rows of P
// of many lengths) is ordered as a whole, since windows pair badly there.
constexpr int kOrderMax = 8192;
constexpr int kOrderKeys = 64;
constexpr int kOrderFewKeys = 8;
__global__ __launch_bounds__(kTileBlock) void k_tile_order(const int* __restrict__ tiles,
                                                           const int* __restrict__ fptr, int* fine,
                                                           const int* __restrict__ P_rowptr,
                                                           const int* __restrict__ P_col,
                                                           const int* __restrict__ slot) {
  __shared__ int rows_l[kOrderMax];
  __shared__ unsigned char key_l[kOrderMax];
  __shared__ int hist[kOrderKeys];
  __shared__ int woff[kOrderKeys];                  // where each key's rows start in the window
  __shared__ int wcnt[kTileBlock / WAVE][kOrderKeys];  // rows per key of each wavefront's lanes
  static_assert(kOrderKeys == WAVE, "the key offsets are scanned by one wavefront");
  static_assert(kTileBlock / WAVE * kOrderKeys == kTileBlock, "one count cleared per thread");
  const int tile = tiles[blockIdx.x];
  const int f0 = fptr[tile], nf = fptr[tile + 1] - f0;
  if (nf < 2 || nf > kOrderMax) return;
  const int wv = threadIdx.x / WAVE;
  if (threadIdx.x < kOrderKeys) hist[threadIdx.x] = 0;
  (&wcnt[0][0])[threadIdx.x] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < nf; q += kTileBlock) {
    const int I = fine[f0 + q];
    int own = 0;
    for (int e = P_rowptr[I]; e < P_rowptr[I + 1]; ++e)
      own += (slot[P_col[e]] >> kTileRowBits) == tile ? 1 : 0;
    const int k = min(own, kOrderKeys - 1);
    rows_l[q] = I;
    key_l[q] = (unsigned char)k;
    atomicAdd(hist + k, 1);
  }
  __syncthreads();
  // With few distinct counts, windows of kTileBlock consecutive rows already pair like with like
  // and keep neighbouring rows together (less re-fetching between sweeps); otherwise the whole
  // tile is one window.
  int nbins = 0;
  for (int v = 0; v < kOrderKeys; ++v) nbins += hist[v] > 0 ? 1 : 0;
  const int win = nbins <= kOrderFewKeys ? kTileBlock : nf;
  // A stable counting sort of each window by key: the window's rows of key v follow those of
  // smaller keys, in list order.  Per chunk of kTileBlock rows, a lane's rank among the earlier
  // lanes of its wavefront with the same key comes from one ballot per distinct key, and the
  // counts of the wavefronts before it from LDS.
  for (int w0 = 0; w0 < nf; w0 += win) {
    const int w1 = min(w0 + win, nf);
    if (threadIdx.x < kOrderKeys) woff[threadIdx.x] = 0;
    __syncthreads();
    for (int q = w0 + threadIdx.x; q < w1; q += kTileBlock) atomicAdd(woff + key_l[q], 1);
    __syncthreads();
    if (wv == 0) {
      const int c = woff[threadIdx.x];
      const int incl = wave_incl_scan(c);
      woff[threadIdx.x] = incl - c;
    }
    __syncthreads();
    for (int base = w0; base < w1; base += kTileBlock) {
      const int q = base + threadIdx.x;
      const bool has = q < w1;
      const int k = has ? key_l[q] : -1;
      unsigned long long left = ballot(has);
      int rank = 0;
      while (left) {  // the same for every lane of the wavefront
        const int leader = __builtin_ctzll(left);
        const int kv = __shfl(k, leader, WAVE);
        const unsigned long long m = ballot(has && k == kv);
        if (has && k == kv) rank = prefix_count(m);
        if (lane() == leader) wcnt[wv][kv] = __popcll(m);
        left &= ~m;
      }
      __syncthreads();
      if (has) {
        int pos = woff[k] + rank;
        for (int w = 0; w < wv; ++w) pos += wcnt[w][k];
        fine[f0 + w0 + pos] = rows_l[q];
      }
      __syncthreads();
      if (threadIdx.x < kOrderKeys) {  // past this chunk's rows; counts cleared for the next
        int add = 0;
        for (int w = 0; w < kTileBlock / WAVE; ++w) {
          add += wcnt[w][threadIdx.x];
          wcnt[w][threadIdx.x] = 0;
        }
        woff[threadIdx.x] += add;
      }
      __syncthreads();
    }
  }
}

hipError_t launch_tile_order(const Patterns& p, const int* tiles, int ntiles, const int* fptr,
                             int* fine, const int* slot, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_order, dim3(ntiles), dim3(kTileBlock), 0, s, tiles, fptr, fine,
                     p.P_rowptr, p.P_col, slot);
  return hipGetLastError();
}

hipError_t launch_tile_fine(const Patterns& p, const int* pt_ptr, const int* pt_row,
                            const TileSet& ts, int ntiles, const int* r, bool fill, int* cnt_out,
                            int* rmax_out, const int* fptr, int* fine, int part, int K,
                            hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fill)
    hipLaunchKernelGGL(k_tile_fine<true>, dim3(ntiles), dim3(kTileBlock), 0, s, pt_ptr, pt_row, ts,
                       r, p.A_rowptr, p.P_rowptr, cnt_out, rmax_out, fptr, fine, part, p.n, p.m, K);
  else
    hipLaunchKernelGGL(k_tile_fine<false>, dim3(ntiles), dim3(kTileBlock), 0, s, pt_ptr, pt_row, ts,
                       r, p.A_rowptr, p.P_rowptr, cnt_out, rmax_out, fptr, fine, part, p.n, p.m, K);
  return hipGetLastError();
}

// =============================================================================================
// Numeric, atomic fold (F1): one wavefront per fine row I in row order.  R_I is formed in a hash
// map (Alg. 3), then for every selected P(I,i) the lanes walk C's column list of row i, look the
// column up in R_I and add P(I,i) * R_I(j) to C at that slot with a device-wide FP64 atomic
// (Eq. allatonceoutproduct, the outer product of row I of P and row I of AP).
// =============================================================================================
template <bool G>
__global__ __launch_bounds__(kThreads) void k_atomic_numeric(NumericArgs a,
                                                             const int* __restrict__ rows,
                                                             int count, int cap, int* gtab,
                                                             double* gval) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem) + wid;
  int* keys;
  double* vals;
  if (G) {
    keys = gtab + (size_t)gw * cap;
    vals = gval + (size_t)gw * cap;
  } else {
    unsigned char* base = smem + kWavesPerBlock * sizeof(WaveScratch);
    vals = reinterpret_cast<double*>(base) + (size_t)wid * cap;
    keys = reinterpret_cast<int*>(base + (size_t)kWavesPerBlock * cap * sizeof(double)) + wid * cap;
  }
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  const Patterns& p = a.p;
  table_clear<G>(keys, vals, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int I = rows[r];
    const int p0 = p.P_rowptr[I], p1 = p.P_rowptr[I + 1];
    bool any = false;
    for (int e = p0 + ln; e < p1; e += WAVE) any |= part_takes(a.part, I, p.P_col[e], p.n, p.m, a.K);
    if (!ballot(any)) continue;  // empty P_o / P_d row: skipped (Alg. 8, 10)
    for_products(p.A_rowptr[I], p.A_rowptr[I + 1], p.A_col, a.A_val, p.P_rowptr, ws,
                 [&](int k, double av) { hm_add<G>(keys, vals, mask, shift, p.P_col[k], av * a.P_val[k]); });
    if constexpr (G) __threadfence();
    for (int pb = p0; pb < p1; pb += WAVE) {
      const int e = pb + ln;
      const bool ok = e < p1 && part_takes(a.part, I, p.P_col[e], p.n, p.m, a.K);
      unsigned long long mk = ballot(ok);
      const int my_i = ok ? p.P_col[e] : 0;
      const double my_w = ok ? a.P_val[e] : 0.0;
      while (mk) {
        const int src = __ffsll((long long)mk) - 1;
        mk &= mk - 1;
        const int i = __shfl(my_i, src, WAVE);
        const double w = __shfl(my_w, src, WAVE);
        for (int c = a.C_rowptr[i] + ln; c < a.C_rowptr[i + 1]; c += WAVE) {
          const int s = hs_find<G>(keys, mask, shift, a.C_col[c]);
          if (s >= 0) unsafeAtomicAdd(a.C_val + c, w * ld_val<G>(vals + s));
        }
      }
    }
    table_clear<G>(keys, vals, cap);
  }
}

static size_t map_lds_bytes(int cap) {
  return kWavesPerBlock * (sizeof(WaveScratch) + (size_t)cap * (sizeof(int) + sizeof(double)));
}

// Numeric cache: for every entry A(I,J) the extent of row J of P, start and length packed as
// (start << 6) | min(length, 63).  Only rows of P with at most 32 entries are read back from it
// (the short-row owner kernel), so the length never saturates where it is used.
__global__ void k_pext(Patterns p, long long nnzA, int* __restrict__ out) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nnzA;
       t += (long long)gridDim.x * blockDim.x) {
    const int J = p.A_col[t];
    const int ps = p.P_rowptr[J], len = p.P_rowptr[J + 1] - ps;
    // unsigned: starts up to 2^26 fill all 32 bits (the sign bit included)
    out[t] = (int)(((unsigned)ps << 6) | (unsigned)(len < 63 ? len : 63));
  }
}

hipError_t launch_pext(const Patterns& p, long long nnzA, int* out, hipStream_t s) {
  if (nnzA == 0) return hipSuccess;
  const long long blocks = std::min<long long>((nnzA + 255) / 256, 65536);
  hipLaunchKernelGGL(k_pext, dim3((unsigned)blocks), dim3(256), 0, s, p, nnzA, out);
  return hipGetLastError();
}

hipError_t launch_atomic_numeric(const NumericArgs& a, const RowClass& rc, int* gtab, double* gval,
                                 hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  if (rc.global)
    hipLaunchKernelGGL(k_atomic_numeric<true>, dim3(grid), dim3(kThreads),
                       kWavesPerBlock * sizeof(WaveScratch), s, a, rc.rows, rc.count, rc.cap, gtab,
                       gval);
  else
    hipLaunchKernelGGL(k_atomic_numeric<false>, dim3(grid), dim3(kThreads), map_lds_bytes(rc.cap), s,
                       a, rc.rows, rc.count, rc.cap, gtab, gval);
  return hipGetLastError();
}

// =============================================================================================
// Numeric, owner fold (F2), general rows: a workgroup owns a tile of rows of C whose values live
// in LDS.  Its wavefronts take the tile's fine rows I in turn, form R_I in a per-wavefront hash
// map, and for every P(I,i) with i in the tile add P(I,i) * R_I(j) into the tile's copy of row i
// (LDS atomics; slots found by walking row i's columns and looking each up in R_I).  The tile is
// written to C once.  No device-wide atomics.  Tables and tiles too large for LDS live in device
// memory (HG, TG).
// =============================================================================================
template <bool HG, bool TG>
__global__ __launch_bounds__(kThreads) void k_owner_numeric(NumericArgs a,
                                                            const int* __restrict__ tiles,
                                                            TileSet ts,
                                                            const int* __restrict__ tile_fptr,
                                                            const int* __restrict__ tile_fine,
                                                            int cap, int TE, int xcd_remap,
                                                            int* gtab, double* gval) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  int b = blockIdx.x;
  if (xcd_remap) {
    // Workgroups are dispatched to the 8 XCDs round-robin; give XCD x a contiguous run of tiles
    // so neighbouring tiles (which share fine rows) meet in the same L2.
    const int T = gridDim.x, q = T / 8, rem = T % 8, x = b % 8, k = b / 8;
    b = x * q + min(x, rem) + k;
  }
  const int tile = tiles[b];
  const int tp = ts.ptr[tile], nr = ts.ptr[tile + 1] - tp;
  const Patterns& p = a.p;

  const host::OwnerLayout lay =
      host::owner_general_layout(TE, cap, kWavesPerBlock, sizeof(WaveScratch), !TG, !HG);
  double* tv;
  const int* tc;
  int* trp = nullptr;
  int tg_len = 0;
  if (TG) {
    // one row longer than a tile: accumulate in C itself (zeroed beforehand)
    const int row = ts.rows[tp];
    const int c0 = a.C_rowptr[row];
    tv = a.C_val + c0;
    tc = a.C_col + c0;
    tg_len = a.C_rowptr[row + 1] - c0;
  } else {
    tv = reinterpret_cast<double*>(smem + lay.tv);
    int* tcw = reinterpret_cast<int*>(smem + lay.tc);
    trp = reinterpret_cast<int*>(smem + lay.trp);
    tile_load(ts.rows, tp, nr, a.C_rowptr, a.C_col, trp, tcw, tv);
    tc = tcw;
  }
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem + lay.ws) + wid;
  int* keys;
  double* vals;
  if (HG) {
    const int gw = blockIdx.x * kWavesPerBlock + wid;
    keys = gtab + (size_t)gw * cap;
    vals = gval + (size_t)gw * cap;
  } else {
    vals = reinterpret_cast<double*>(smem + lay.vals) + (size_t)wid * cap;
    keys = reinterpret_cast<int*>(smem + lay.keys) + (size_t)wid * cap;
  }
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  table_clear<HG>(keys, vals, cap);
  __syncthreads();

  // a.part < 0: the two passes of Alg. 8 (off-block entries, then on-block entries, R_I formed
  // in each; the first pass walks only the tile's rows with off-block entries); otherwise one
  // pass over the given part.
  const int npass = a.part < 0 ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int part = a.part < 0 ? (pass == 0 ? PART_OFF : PART_ON) : a.part;
    const bool off_list = pass == 0 && npass == 2 && a.off_fptr != nullptr;
    const int* fine = off_list ? a.off_fine : tile_fine;
    const int f0 = off_list ? a.off_fptr[tile] : tile_fptr[tile];
    const int f1 = off_list ? a.off_fptr[tile + 1] : tile_fptr[tile + 1];
    for (int f = f0 + wid; f < f1; f += kWavesPerBlock) {
      const int I = fine[f];
      const int p0 = p.P_rowptr[I], p1 = p.P_rowptr[I + 1];
      bool any = false;
      for (int e = p0 + ln; e < p1; e += WAVE) {
        const int i = p.P_col[e];
        any |= (ts.slot[i] >> kTileRowBits) == tile && part_takes(part, I, i, p.n, p.m, a.K);
      }
      if (!ballot(any)) continue;
      for_products(p.A_rowptr[I], p.A_rowptr[I + 1], p.A_col, a.A_val, p.P_rowptr, ws,
                   [&](int k, double av) { hm_add<HG>(keys, vals, mask, shift, p.P_col[k], av * a.P_val[k]); });
      if constexpr (HG) __threadfence();
      for (int pb = p0; pb < p1; pb += WAVE) {
        const int e = pb + ln;
        int my_l = 0;
        bool ok = false;
        if (e < p1) {
          const int i = p.P_col[e];
          const int sl = ts.slot[i];
          ok = (sl >> kTileRowBits) == tile && part_takes(part, I, i, p.n, p.m, a.K);
          my_l = sl & (kTileRows - 1);
        }
        unsigned long long mk = ballot(ok);
        const double my_w = ok ? a.P_val[e] : 0.0;
        while (mk) {
          const int src = __ffsll((long long)mk) - 1;
          mk &= mk - 1;
          const int il = __shfl(my_l, src, WAVE);
          const double w = __shfl(my_w, src, WAVE);
          const int cb = TG ? 0 : trp[il];
          const int ce = TG ? tg_len : trp[il + 1];
          for (int c = cb + ln; c < ce; c += WAVE) {
            const int s = hs_find<HG>(keys, mask, shift, tc[c]);
            if (s >= 0) {
              if (TG)
                unsafeAtomicAdd(tv + c, w * ld_val<HG>(vals + s));
              else
                atomicAdd(tv + c, w * ld_val<HG>(vals + s));
            }
          }
        }
      }
      table_clear<HG>(keys, vals, cap);
    }
  }
  if (!TG) {
    __syncthreads();
    tile_store(ts.rows, tp, nr, a.C_rowptr, trp, tv, a.C_val);
  }
}

size_t owner_general_lds_bytes(int TE, int cap, bool hash_global, bool tile_global) {
  return host::owner_general_layout(TE, cap, kWavesPerBlock, sizeof(WaveScratch), !tile_global, !hash_global)
      .total;
}

hipError_t launch_owner_numeric(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                                const int* tile_fptr, const int* tile_fine, int tile_entries,
                                bool xcd_remap, int* gtab, double* gval, hipStream_t s) {
  if (tc.count == 0) return hipSuccess;
  const size_t lds = owner_general_lds_bytes(tile_entries, tc.cap, tc.hash_global, tc.tile_global);
  // Spill tables are indexed by workgroup, so a spill class launches exactly its tiles and the
  // workspace holds one table per wavefront of the largest spill class.
  const int grid = tc.count;
  const int remap = xcd_remap ? 1 : 0;
#define PTAP_LAUNCH_OWN(HG, TG)                                                                \
  hipLaunchKernelGGL((k_owner_numeric<HG, TG>), dim3(grid), dim3(kThreads), lds, s, a, tc.tiles, \
                     ts, tile_fptr, tile_fine, tc.cap, tile_entries, remap, gtab, gval)
  if (tc.hash_global) {
    if (tc.tile_global) PTAP_LAUNCH_OWN(true, true); else PTAP_LAUNCH_OWN(true, false);
  } else {
    if (tc.tile_global) PTAP_LAUNCH_OWN(false, true); else PTAP_LAUNCH_OWN(false, false);
  }
#undef PTAP_LAUNCH_OWN
  return hipGetLastError();
}

// =============================================================================================
// Two-step numeric (Alg. 6): stored AP by rows (Alg. 4), the values of the explicit transpose
// of P, and C = P^T (AP) by rows of P^T.
// =============================================================================================
template <bool G>
__global__ __launch_bounds__(kThreads) void k_ap_numeric(NumericArgs a, const int* __restrict__ rows,
                                                         int count, int cap,
                                                         const int* __restrict__ AP_rowptr,
                                                         const int* __restrict__ AP_col,
                                                         double* AP_val, int* gtab, double* gval) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem) + wid;
  int* keys;
  double* vals;
  if (G) {
    keys = gtab + (size_t)gw * cap;
    vals = gval + (size_t)gw * cap;
  } else {
    unsigned char* base = smem + kWavesPerBlock * sizeof(WaveScratch);
    vals = reinterpret_cast<double*>(base) + (size_t)wid * cap;
    keys = reinterpret_cast<int*>(base + (size_t)kWavesPerBlock * cap * sizeof(double)) + wid * cap;
  }
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  const Patterns& p = a.p;
  table_clear<G>(keys, vals, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int I = rows[r];
    for_products(p.A_rowptr[I], p.A_rowptr[I + 1], p.A_col, a.A_val, p.P_rowptr, ws,
                 [&](int k, double av) { hm_add<G>(keys, vals, mask, shift, p.P_col[k], av * a.P_val[k]); });
    if constexpr (G) __threadfence();
    for (int e = AP_rowptr[I] + ln; e < AP_rowptr[I + 1]; e += WAVE) {
      const int sl = hs_find<G>(keys, mask, shift, AP_col[e]);
      AP_val[e] = sl >= 0 ? ld_val<G>(vals + sl) : 0.0;
    }
    table_clear<G>(keys, vals, cap);
  }
}

hipError_t launch_ap_numeric(const NumericArgs& a, const RowClass& rc, const int* AP_rowptr,
                             const int* AP_col, double* AP_val, int* gtab, double* gval,
                             hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  if (rc.global)
    hipLaunchKernelGGL(k_ap_numeric<true>, dim3(grid), dim3(kThreads),
                       kWavesPerBlock * sizeof(WaveScratch), s, a, rc.rows, rc.count, rc.cap,
                       AP_rowptr, AP_col, AP_val, gtab, gval);
  else
    hipLaunchKernelGGL(k_ap_numeric<false>, dim3(grid), dim3(kThreads), map_lds_bytes(rc.cap), s, a,
                       rc.rows, rc.count, rc.cap, AP_rowptr, AP_col, AP_val, gtab, gval);
  return hipGetLastError();
}

__global__ void k_gather(const double* __restrict__ src, const int* __restrict__ idx,
                         double* __restrict__ dst, long long count) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < count;
       k += (long long)gridDim.x * blockDim.x)
    dst[k] = src[idx[k]];
}

hipError_t launch_gather(const double* src, const int* idx, double* dst, long long count,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, src, idx, dst,
                     count);
  return hipGetLastError();
}

template <bool G>
__global__ __launch_bounds__(kThreads) void k_ptc_numeric(
    const int* __restrict__ pt_ptr, const int* __restrict__ pt_row,
    const double* __restrict__ PT_val, const int* __restrict__ AP_rowptr,
    const int* __restrict__ AP_col, const double* __restrict__ AP_val,
    const int* __restrict__ C_rowptr, const int* __restrict__ C_col, double* C_val,
    const int* __restrict__ rows, int count, int cap, int* gtab, double* gval) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  int* keys;
  double* vals;
  if (G) {
    keys = gtab + (size_t)gw * cap;
    vals = gval + (size_t)gw * cap;
  } else {
    vals = reinterpret_cast<double*>(smem) + (size_t)wid * cap;
    keys = reinterpret_cast<int*>(smem + (size_t)kWavesPerBlock * cap * sizeof(double)) + wid * cap;
  }
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  table_clear<G>(keys, vals, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int i = rows[r];
    for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) {
      const int I = pt_row[t];
      const double w = PT_val[t];
      for (int e = AP_rowptr[I] + ln; e < AP_rowptr[I + 1]; e += WAVE)
        hm_add<G>(keys, vals, mask, shift, AP_col[e], w * AP_val[e]);
    }
    if constexpr (G) __threadfence();
    for (int c = C_rowptr[i] + ln; c < C_rowptr[i + 1]; c += WAVE) {
      const int sl = hs_find<G>(keys, mask, shift, C_col[c]);
      C_val[c] = sl >= 0 ? ld_val<G>(vals + sl) : 0.0;
    }
    table_clear<G>(keys, vals, cap);
  }
}

hipError_t launch_ptc_numeric(const int* pt_ptr, const int* pt_row, const double* PT_val,
                              const int* AP_rowptr, const int* AP_col, const double* AP_val,
                              const int* C_rowptr, const int* C_col, double* C_val,
                              const RowClass& rc, int* gtab, double* gval, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  const size_t lds = rc.global ? 0 : (size_t)kWavesPerBlock * rc.cap * (sizeof(int) + sizeof(double));
  if (rc.global)
    hipLaunchKernelGGL(k_ptc_numeric<true>, dim3(grid), dim3(kThreads), lds, s, pt_ptr, pt_row,
                       PT_val, AP_rowptr, AP_col, AP_val, C_rowptr, C_col, C_val, rc.rows, rc.count,
                       rc.cap, gtab, gval);
  else
    hipLaunchKernelGGL(k_ptc_numeric<false>, dim3(grid), dim3(kThreads), lds, s, pt_ptr, pt_row,
                       PT_val, AP_rowptr, AP_col, AP_val, C_rowptr, C_col, C_val, rc.rows, rc.count,
                       rc.cap, gtab, gval);
  return hipGetLastError();
}

// =============================================================================================
// Adjoint (dL/dA and dL/dP of L with dL/dC = dC), one wavefront per fine row I:
//   U_I = sum_{i in P(I,:)} P(I,i) dC(i,:)           (hash map over coarse columns j)
//   R_I = A(I,:) P                                   (hash map, formed again)
//   for each product (J, j) of row I:  dA(I,J) += U_I(j) P(J,j),  dP(J,j) += A(I,J) U_I(j)
//   for each P(I,k): dP(I,k) += sum_j R_I(j) dC(k,j)  (walk C's row k, look up R_I)
// which are the entries of P dC P^T on A's pattern and of A P dC^T + A^T P dC on P's pattern.
// dP must be zeroed first (it receives device-wide atomic adds).
// =============================================================================================
template <bool G>
__global__ __launch_bounds__(kThreads) void k_backward(NumericArgs a, const double* __restrict__ dC,
                                                       double* dA, double* dP,
                                                       const int* __restrict__ rows, int count,
                                                       int cap, int* gtab, double* gval) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  WaveScratch* ws = reinterpret_cast<WaveScratch*>(smem) + wid;
  double* dacc = reinterpret_cast<double*>(smem + kWavesPerBlock * sizeof(WaveScratch)) + wid * WAVE;
  int *ukeys, *rkeys;
  double *uvals, *rvals;
  if (G) {
    ukeys = gtab + (size_t)gw * 2 * cap;
    rkeys = ukeys + cap;
    uvals = gval + (size_t)gw * 2 * cap;
    rvals = uvals + cap;
  } else {
    unsigned char* base = smem + kWavesPerBlock * (sizeof(WaveScratch) + WAVE * sizeof(double));
    uvals = reinterpret_cast<double*>(base) + (size_t)wid * 2 * cap;
    rvals = uvals + cap;
    ukeys = reinterpret_cast<int*>(base + (size_t)kWavesPerBlock * 2 * cap * sizeof(double)) +
            wid * 2 * cap;
    rkeys = ukeys + cap;
  }
  const unsigned mask = (unsigned)cap - 1;
  const int shift = 32 - log2_pow2(cap);
  const Patterns& p = a.p;
  table_clear<G>(ukeys, uvals, cap);
  table_clear<G>(rkeys, rvals, cap);
  for (int r = gw; r < count; r += gridDim.x * kWavesPerBlock) {
    const int I = rows[r];
    const int p0 = p.P_rowptr[I], p1 = p.P_rowptr[I + 1];
    const int a0 = p.A_rowptr[I], a1 = p.A_rowptr[I + 1];
    // U_I
    for (int e = p0; e < p1; ++e) {
      const int i = p.P_col[e];
      const double w = a.P_val[e];
      for (int c = a.C_rowptr[i] + ln; c < a.C_rowptr[i + 1]; c += WAVE)
        hm_add<G>(ukeys, uvals, mask, shift, a.C_col[c], w * dC[c]);
    }
    // R_I (only needed for the dP term of row I)
    if (dP && p1 > p0)
      for_products(a0, a1, p.A_col, a.A_val, p.P_rowptr, ws,
                   [&](int k, double av) { hm_add<G>(rkeys, rvals, mask, shift, p.P_col[k], av * a.P_val[k]); });
    if constexpr (G) __threadfence();
    // products (J, j): dA(I,J) and the A^T P dC part of dP
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
      const int incl = wave_incl_scan(pl);
      const int total = __shfl(incl, WAVE - 1, WAVE);
      ws->off[ln] = incl - pl;
      ws->ps[ln] = ps;
      ws->a[ln] = av;
      dacc[ln] = 0.0;
      wave_sync();
      for (int q = ln; q < total; q += WAVE) {
        int lo = 0;
#pragma unroll
        for (int step = WAVE / 2; step > 0; step >>= 1)
          if (ws->off[lo + step] <= q) lo += step;
        const int k = ws->ps[lo] + (q - ws->off[lo]);
        const int s = hs_find<G>(ukeys, mask, shift, p.P_col[k]);
        if (s >= 0) {
          const double u = ld_val<G>(uvals + s);
          atomicAdd(dacc + lo, u * a.P_val[k]);
          if (dP) unsafeAtomicAdd(dP + k, ws->a[lo] * u);
        }
      }
      wave_sync();
      if (dA && t < a1) dA[t] = dacc[ln];
      wave_sync();
    }
    // A P dC^T part of dP: dP(I,k) += sum_j R_I(j) dC(k,j)
    if (dP) {
      for (int e = p0; e < p1; ++e) {
        const int k = p.P_col[e];
        double sum = 0.0;
        for (int c = a.C_rowptr[k] + ln; c < a.C_rowptr[k + 1]; c += WAVE) {
          const int s = hs_find<G>(rkeys, mask, shift, a.C_col[c]);
          if (s >= 0) sum += ld_val<G>(rvals + s) * dC[c];
        }
        sum = wave_sum(sum);
        if (ln == 0) unsafeAtomicAdd(dP + e, sum);
      }
    }
    table_clear<G>(ukeys, uvals, cap);
    table_clear<G>(rkeys, rvals, cap);
  }
}

hipError_t launch_backward(const NumericArgs& a, const double* dC, double* dA, double* dP,
                           const RowClass& rc, int* gtab, double* gval, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  const int grid = wave_grid(rc.count, rc.global);
  size_t lds = kWavesPerBlock * (sizeof(WaveScratch) + WAVE * sizeof(double));
  if (!rc.global) lds += (size_t)kWavesPerBlock * 2 * rc.cap * (sizeof(int) + sizeof(double));
  if (rc.global)
    hipLaunchKernelGGL(k_backward<true>, dim3(grid), dim3(kThreads), lds, s, a, dC, dA, dP, rc.rows,
                       rc.count, rc.cap, gtab, gval);
  else
    hipLaunchKernelGGL(k_backward<false>, dim3(grid), dim3(kThreads), lds, s, a, dC, dA, dP, rc.rows,
                       rc.count, rc.cap, gtab, gval);
  return hipGetLastError();
}

}  // namespace ptapk
