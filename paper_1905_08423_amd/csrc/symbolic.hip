// Device building blocks of the symbolic phase (Section 3, Alg. 7 / Alg. 9: the pattern of C is
// found without storing AP): exclusive prefix sums, row classes by a stable counting sort, a
// validation pass over the input patterns, |R_I| together with the product counts w_I, the
// pattern of C by a two-level union, and the per-row codes that sort rows into launch classes.
// Everything here runs on the device; the host reads back only a few counters.
#include "device.hpp"
#include "host_logic.hpp"
#include "internal.hpp"

namespace ptapk {

namespace {

constexpr int kSymBlock = 256;                       // threads per workgroup of these kernels
constexpr int kSymWaves = kSymBlock / WAVE;
constexpr int kScanItems = 8;                        // items per thread of a scan workgroup
constexpr int kScanChunk = kSymBlock * kScanItems;  // items per scan workgroup

inline int blocks_for(long long count, int per_block) {
  long long g = (count + per_block - 1) / per_block;
  return (int)(g < 1 ? 1 : g);
}

// Exclusive scan of one value per thread over a kSymBlock workgroup; `red` holds kSymWaves
// entries.  Returns this thread's offset and the workgroup total.
template <class T>
__device__ __forceinline__ T block_scan(T v, T* red, T& total) {
  const int ln = lane(), wid = threadIdx.x / WAVE;
  T incl = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const T t = __shfl_up(incl, d, WAVE);
    if (ln >= d) incl += t;
  }
  if (ln == WAVE - 1) red[wid] = incl;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kSymWaves; ++w) {
    if (w < wid) before += red[w];
    tot += red[w];
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

template <class T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  T total;
  (void)block_scan(v, red, total);
  return total;
}

// Device twin of host::cap_log2: log2 of the hash capacity for a row with at most `need` keys.
__device__ __forceinline__ int dev_cap_log2(long long need) {
  const unsigned long long v = 2ULL * (unsigned long long)need;
  const int b = v <= 64 ? 6 : 64 - __clzll((long long)(v - 1));
  return b < 30 ? b : 30;
}

}  // namespace

// =============================================================================================
// Exclusive prefix sum of int counts: out[k] = in[0] + ... + in[k-1] for k = 0..n, so out[n] is
// the total.  Three passes: workgroup sums, a scan of those sums in one workgroup, and the
// workgroup-local scans.  A total beyond INT32_MAX sets *flag (out is then not usable); the
// total is also written as a 64-bit value to *total64.
// =============================================================================================
__global__ __launch_bounds__(kSymBlock) void k_scan_reduce(const int* __restrict__ in, long long n,
                                                           long long* bsum) {
  __shared__ long long red[kSymWaves];
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanItems;
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) s += in[base + j];
  s = block_sum(s, red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kSymBlock) void k_scan_top(long long* bsum, long long nb, int* out,
                                                        long long n, long long* total64, int* flag) {
  __shared__ long long red[kSymWaves];
  long long carry = 0;
  for (long long b0 = 0; b0 < nb; b0 += kSymBlock) {
    const long long b = b0 + threadIdx.x;
    const long long v = b < nb ? bsum[b] : 0;
    long long tot;
    const long long ex = block_scan(v, red, tot);
    if (b < nb) bsum[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *total64 = carry;
    if (carry > (long long)INT32_MAX) atomicOr(flag, 1);
    out[n] = (int)(carry > (long long)INT32_MAX ? INT32_MAX : carry);
  }
}

__global__ __launch_bounds__(kSymBlock) void k_scan_down(const int* __restrict__ in, long long n,
                                                         const long long* __restrict__ boff, int* out) {
  __shared__ long long red[kSymWaves];
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  long long tot;
  long long run = boff[blockIdx.x] + block_scan(s, red, tot);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = (int)(run > (long long)INT32_MAX ? INT32_MAX : run);
    run += v[j];
  }
}

size_t scan_scratch_count(long long n) { return (size_t)blocks_for(n, kScanChunk) + 1; }

hipError_t launch_scan_i32(const int* in, long long n, int* out, long long* scratch, int* flag,
                           hipStream_t s) {
  const int nb = blocks_for(n, kScanChunk);
  long long* total64 = scratch + nb;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kSymBlock), 0, s, in, n, scratch);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSymBlock), 0, s, scratch, (long long)nb, out, n, total64,
                     flag);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kSymBlock), 0, s, in, n, scratch, out);
  return hipGetLastError();
}

// =============================================================================================
// Row classes by a stable counting sort.  Item k (k = 0..count-1) stands for row list[k] (or k
// without a list) and carries code[k] in [0, nbins) or a negative code (dropped).  The rows come
// out grouped by code, each group in ascending item order, in `sorted`; hist[b] is the size of
// group b, whose rows start at hist[0] + ... + hist[b-1].
//   pass 1: per workgroup and code, the count of its items (bin-major: blk[b * nblk + g]);
//   pass 2: an exclusive scan of those counts gives each (code, workgroup) its output start;
//   pass 3: each workgroup ranks its items within each code present (ballots) and writes them.
// =============================================================================================
__global__ __launch_bounds__(kSymBlock) void k_class_count(const int* __restrict__ code, int count,
                                                           int nbins, int* blk, int nblk) {
  __shared__ int c[kMaxClassBins];
  for (int b = threadIdx.x; b < nbins; b += kSymBlock) c[b] = 0;
  __syncthreads();
  const long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  if (k < count) {
    const int b = code[k];
    if (b >= 0) atomicAdd(c + b, 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kSymBlock) blk[(long long)b * nblk + blockIdx.x] = c[b];
}

__global__ __launch_bounds__(kSymBlock) void k_class_scatter(const int* __restrict__ code,
                                                             const int* __restrict__ list, int count,
                                                             const int* __restrict__ pos, int nblk,
                                                             int* sorted) {
  __shared__ unsigned present[kMaxClassBins / 32];
  __shared__ int wtot[kSymWaves];
  const int wid = threadIdx.x / WAVE;
  for (int w = threadIdx.x; w < kMaxClassBins / 32; w += kSymBlock) present[w] = 0u;
  __syncthreads();
  const long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  const int b = k < count ? code[k] : -1;
  if (b >= 0) atomicOr(present + (b >> 5), 1u << (b & 31));
  __syncthreads();
  for (int w = 0; w < kMaxClassBins / 32; ++w) {
    unsigned bits = present[w];  // the same for every thread: the loop is uniform
    while (bits) {
      const int bin = w * 32 + __ffs(bits) - 1;
      bits &= bits - 1;
      const unsigned long long mk = ballot(b == bin);
      if (lane() == 0) wtot[wid] = __popcll(mk);
      __syncthreads();
      int before = 0;
      for (int q = 0; q < wid; ++q) before += wtot[q];
      if (b == bin)
        sorted[pos[(long long)bin * nblk + blockIdx.x] + before + prefix_count(mk)] = list ? list[k] : (int)k;
      __syncthreads();
    }
  }
}

__global__ void k_class_hist(const int* __restrict__ pos, int nbins, int nblk, int* hist) {
  const int b = threadIdx.x;
  if (b < nbins) hist[b] = pos[(long long)(b + 1) * nblk] - pos[(long long)b * nblk];
}

size_t class_scratch_ints(int count, int nbins) {
  return (size_t)nbins * (size_t)blocks_for(count, kSymBlock) + 1;
}

hipError_t launch_class_build(const int* code, const int* list, int count, int nbins, int* scratch,
                              long long* scan_scratch, int* flag, int* sorted, int* hist, hipStream_t s) {
  if (nbins < 1 || nbins > kMaxClassBins) return hipErrorInvalidValue;
  const int nblk = blocks_for(count, kSymBlock);
  hipLaunchKernelGGL(k_class_count, dim3(nblk), dim3(kSymBlock), 0, s, code, count, nbins, scratch, nblk);
  const long long cells = (long long)nbins * nblk;
  // the scan runs in place: out may alias in because each workgroup reads its chunk before it
  // writes it and the chunks are disjoint
  hipError_t e = launch_scan_i32(scratch, cells, scratch, scan_scratch, flag, s);
  if (e != hipSuccess) return e;
  if (count > 0)
    hipLaunchKernelGGL(k_class_scatter, dim3(nblk), dim3(kSymBlock), 0, s, code, list, count, scratch, nblk,
                       sorted);
  hipLaunchKernelGGL(k_class_hist, dim3(1), dim3(kMaxClassBins), 0, s, scratch, nbins, nblk, hist);
  return hipGetLastError();
}

// Codes by hash capacity: log2 of the capacity for need[row] keys, or -1 for need <= 0.
template <class T>
__global__ void k_cap_codes(const T* __restrict__ need, const int* __restrict__ list, int count, int* code) {
  const long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  if (k >= count) return;
  const long long v = (long long)need[list ? list[k] : (int)k];
  code[k] = v <= 0 ? -1 : dev_cap_log2(v);
}

hipError_t launch_cap_codes_i32(const int* need, const int* list, int count, int* code, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cap_codes<int>, dim3(blocks_for(count, kSymBlock)), dim3(kSymBlock), 0, s, need, list,
                     count, code);
  return hipGetLastError();
}

hipError_t launch_cap_codes_i64(const long long* need, const int* list, int count, int* code, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cap_codes<long long>, dim3(blocks_for(count, kSymBlock)), dim3(kSymBlock), 0, s, need,
                     list, count, code);
  return hipGetLastError();
}

// =============================================================================================
// Validation of a CSR pattern (row pointers from 0 to nnz, non-decreasing; columns in range and
// strictly increasing within each row), one thread per row and one per entry.  A strict
// increase is checked by counting descents col[k] <= col[k-1] over all of col and over the
// first entries of non-empty rows only: once the row pointers are valid, the columns are
// sorted within rows exactly when every descent falls on a row start, that is when the two
// counts agree.  cnt[0] counts descents at row starts, cnt[1] all descents.
//   err bit 1: rowptr[0] != 0 or rowptr[nrows] != nnz; bit 2: a row's extent is out of range
//   or decreasing; bit 4: a column out of range.
// =============================================================================================
__global__ __launch_bounds__(kSymBlock) void k_validate_rows(const int* __restrict__ rowptr,
                                                             const int* __restrict__ col, int nrows,
                                                             long long nnz, int* err,
                                                             unsigned long long* cnt) {
  __shared__ unsigned long long red[kSymWaves];
  unsigned long long d = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rowptr[0] != 0 || (long long)rowptr[nrows] != nnz))
    atomicOr(err, 1);
  for (long long r = (long long)blockIdx.x * kSymBlock + threadIdx.x; r < nrows;
       r += (long long)gridDim.x * kSymBlock) {
    const long long b = rowptr[r], e = rowptr[r + 1];
    if (b < 0 || e < b || e > nnz) {
      atomicOr(err, 2);
      continue;
    }
    if (e > b && b >= 1) d += col[b] <= col[b - 1] ? 1 : 0;
  }
  d = block_sum(d, red);
  if (threadIdx.x == 0 && d) atomicAdd(cnt, d);
}

__global__ __launch_bounds__(kSymBlock) void k_validate_cols(const int* __restrict__ col, long long nnz,
                                                             int ncols, int* err, unsigned long long* cnt) {
  __shared__ unsigned long long red[kSymWaves];
  unsigned long long d = 0;
  bool bad = false;
  for (long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x; k < nnz;
       k += (long long)gridDim.x * kSymBlock) {
    const int c = col[k];
    bad = bad || c < 0 || c >= ncols;
    if (k >= 1) d += c <= col[k - 1] ? 1 : 0;
  }
  if (bad) atomicOr(err, 4);
  d = block_sum(d, red);
  if (threadIdx.x == 0 && d) atomicAdd(cnt + 1, d);
}

hipError_t launch_validate_pattern(const int* rowptr, const int* col, int nrows, int ncols, long long nnz,
                                   int* err, unsigned long long* cnt, hipStream_t s) {
  constexpr int kMaxBlocks = 2048;  // grid-stride: few workgroup atomics on the counters
  hipLaunchKernelGGL(k_validate_rows, dim3(std::min(blocks_for((long long)nrows + 1, kSymBlock), kMaxBlocks)),
                     dim3(kSymBlock), 0, s, rowptr, col, nrows, nnz, err, cnt);
  if (nnz > 0)
    hipLaunchKernelGGL(k_validate_cols, dim3(std::min(blocks_for(nnz, kSymBlock), kMaxBlocks)), dim3(kSymBlock),
                       0, s, col, nnz, ncols, err, cnt);
  return hipGetLastError();
}

// =============================================================================================
// |R_I| and w_I in one pass (Alg. 1 / Alg. 2): one wavefront per fine row I forms the key set of
// row I of AP in an LDS table of kApCap slots.  w_I, the number of products A(I,J) P(J,j), bounds
// |R_I|; a row with w_I above kApMaxW could overflow the table and is listed in `ovf` instead
// (its |R_I| comes from the launches by capacity class).  w[I] = min(w_I, m).
// =============================================================================================
constexpr int kApCap = 256;
constexpr int kApMaxW = kApCap - WAVE - 1;

__global__ __launch_bounds__(kSymBlock) void k_ap_count(Patterns p, int* r, int* w, int* ovf, int* novf) {
  __shared__ WaveScratch wsa[kSymWaves];
  __shared__ int keys_all[kSymWaves][kApCap];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const long long I64 = (long long)blockIdx.x * kSymWaves + wid;
  if (I64 >= p.n) return;  // uniform over the wavefront
  const int I = (int)I64;
  WaveScratch* ws = wsa + wid;
  int* keys = keys_all[wid];
  const int a0 = p.A_rowptr[I], a1 = p.A_rowptr[I + 1];
  long long prod = 0;
  for (int k = a0 + ln; k < a1; k += WAVE) {
    const int J = p.A_col[k];
    prod += p.P_rowptr[J + 1] - p.P_rowptr[J];
  }
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) prod += __shfl_xor(prod, d, WAVE);
  if (ln == 0) w[I] = (int)(prod < p.m ? prod : p.m);
  if (prod > kApMaxW) {
    if (ln == 0) {
      r[I] = 0;
      ovf[atomicAdd(novf, 1)] = I;
    }
    return;
  }
  for (int q = ln; q < kApCap; q += WAVE) keys[q] = EMPTY;
  wave_sync();
  constexpr unsigned mask = kApCap - 1;
  constexpr int shift = 32 - 8;  // log2(kApCap) = 8
  static_assert(kApCap == 256, "shift assumes 256 slots");
  int fresh_cnt = 0;
  for_products(a0, a1, p.A_col, nullptr, p.P_rowptr, ws, [&](int k, double) {
    bool fresh;
    hs_insert<false>(keys, mask, shift, p.P_col[k], fresh);
    fresh_cnt += fresh ? 1 : 0;
  });
  fresh_cnt = wave_sum(fresh_cnt);
  if (ln == 0) r[I] = fresh_cnt;
}

hipError_t launch_ap_count(const Patterns& p, int* r, int* w, int* ovf, int* novf, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ap_count, dim3(blocks_for(p.n, kSymWaves)), dim3(kSymBlock), 0, s, p, r, w, ovf, novf);
  return hipGetLastError();
}

// =============================================================================================
// Pattern of C by a two-level union (Eq. allatoncerow): C(i,:) is the union over I with P(I,i)
// stored of the union over J in A(I,:) of P(J,:), so with S_i the set of all such J,
// C(i,:) = union over J in S_i of P(J,:).  One wavefront per row i builds S_i in an LDS table,
// then C(i,:) in a second one: neighbouring fine rows I share most of their J, so each distinct
// J is walked once instead of once per I.  A row whose S_i or C(i,:) outgrows its table is
// flagged and listed in `ovf` (count pass) and left to the launches by capacity class; a table
// is checked after every step of 64 inserts and holds at most (capacity - 65) keys before a
// step, so probing always finds a free slot.  Count pass: cnt[i] = |C(i,:)|.  Fill pass: the
// sorted columns at C_rowptr[i], for rows not flagged.
// =============================================================================================
constexpr int kTwoSCap = 512, kTwoSMax = kTwoSCap - WAVE - 1;
constexpr int kTwoCCap = 256, kTwoCMax = kTwoCCap - WAVE - 1;

struct TwoLevelScratch {
  int off[WAVE];
  int st[WAVE];
  int skeys[kTwoSCap];
  int slist[kTwoSMax + 1];
  int ckeys[kTwoCCap];
  int clist[kTwoCMax + 1];
};

// Flattened walk over the entries of nl rows: row x of the list spans [start, start + len) of
// `col` (row_of(x, start, len)); f(key) for each entry, 64 entries per step.  After each step
// the count of new keys (ballot over the lanes' `fresh`) is added to *occ; the walk stops and
// returns false as soon as *occ exceeds `limit`.
template <class RowOf, class F>
__device__ __forceinline__ bool walk_insert(int nl, RowOf row_of, const int* __restrict__ col, int* off,
                                            int* st, int& occ, int limit, F&& insert) {
  const int ln = lane();
  for (int base = 0; base < nl; base += WAVE) {
    int s = 0, l = 0;
    if (base + ln < nl) row_of(base + ln, s, l);
    const int incl = wave_incl_scan(l);
    const int total = __shfl(incl, WAVE - 1, WAVE);
    off[ln] = incl - l;
    st[ln] = s;
    wave_sync();
    for (int q0 = 0; q0 < total; q0 += WAVE) {
      const int q = q0 + ln;
      bool fresh = false;
      if (q < total) {
        int lo = 0;
#pragma unroll
        for (int step = WAVE / 2; step > 0; step >>= 1)
          if (off[lo + step] <= q) lo += step;
        fresh = insert(col[st[lo] + (q - off[lo])]);
      }
      occ += __popcll(ballot(fresh));
      if (occ > limit) {
        wave_sync();
        return false;
      }
    }
    wave_sync();
  }
  return true;
}

template <bool FILL>
__global__ __launch_bounds__(kSymBlock) void k_c_two_level(Patterns p, const int* __restrict__ pt_ptr,
                                                           const int* __restrict__ pt_row, int* cnt,
                                                           unsigned char* flag, int* ovf, int* novf,
                                                           const int* __restrict__ C_rowptr, int* C_col) {
  __shared__ TwoLevelScratch scr[kSymWaves];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const long long i64 = (long long)blockIdx.x * kSymWaves + wid;
  if (i64 >= p.m) return;  // uniform over the wavefront
  const int i = (int)i64;
  if (FILL && flag[i]) return;
  TwoLevelScratch& sc = scr[wid];
  for (int q = ln; q < kTwoSCap; q += WAVE) sc.skeys[q] = EMPTY;
  for (int q = ln; q < kTwoCCap; q += WAVE) sc.ckeys[q] = EMPTY;
  wave_sync();
  constexpr int sshift = 32 - 9, cshift = 32 - 8;
  static_assert(kTwoSCap == 512 && kTwoCCap == 256, "shifts assume these capacities");
  // level 1: S_i from the rows of A under the fine rows I of column i of P
  const int t0 = pt_ptr[i], t1 = pt_ptr[i + 1];
  int ns = 0;
  bool ok = walk_insert(
      t1 - t0,
      [&](int x, int& s, int& l) {
        const int I = pt_row[t0 + x];
        s = p.A_rowptr[I];
        l = p.A_rowptr[I + 1] - s;
      },
      p.A_col, sc.off, sc.st, ns, kTwoSMax,
      [&](int key) {
        bool fresh;
        hs_insert<false>(sc.skeys, kTwoSCap - 1, sshift, key, fresh);
        return fresh;
      });
  int nc = 0;
  if (ok) {
    // S_i as a list
    int base = 0;
    for (int s0 = 0; s0 < kTwoSCap; s0 += WAVE) {
      const int k = sc.skeys[s0 + ln];
      const unsigned long long mk = ballot(k != EMPTY);
      if (k != EMPTY) sc.slist[base + prefix_count(mk)] = k;
      base += __popcll(mk);
    }
    wave_sync();
    // level 2: C(i,:) from the rows of P under S_i
    ok = walk_insert(
        ns,
        [&](int x, int& s, int& l) {
          const int J = sc.slist[x];
          s = p.P_rowptr[J];
          l = p.P_rowptr[J + 1] - s;
        },
        p.P_col, sc.off, sc.st, nc, kTwoCMax,
        [&](int key) {
          bool fresh;
          hs_insert<false>(sc.ckeys, kTwoCCap - 1, cshift, key, fresh);
          return fresh;
        });
  }
  if constexpr (!FILL) {
    if (ln == 0) {
      cnt[i] = ok ? nc : 0;
      flag[i] = ok ? 0 : 1;
      if (!ok) ovf[atomicAdd(novf, 1)] = i;
    }
  } else {
    if (!ok) return;  // not reached for rows the count pass kept
    int base = 0;
    for (int s0 = 0; s0 < kTwoCCap; s0 += WAVE) {
      const int k = sc.ckeys[s0 + ln];
      const unsigned long long mk = ballot(k != EMPTY);
      if (k != EMPTY) sc.clist[base + prefix_count(mk)] = k;
      base += __popcll(mk);
    }
    wave_sync();
    int* out = C_col + C_rowptr[i];
    for (int x = ln; x < base; x += WAVE) {
      const int key = sc.clist[x];
      int rank = 0;
      for (int y = 0; y < base; ++y) rank += sc.clist[y] < key;
      out[rank] = key;
    }
  }
}

hipError_t launch_c_two_level(const Patterns& p, const int* pt_ptr, const int* pt_row, bool fill, int* cnt,
                              unsigned char* flag, int* ovf, int* novf, const int* C_rowptr, int* C_col,
                              hipStream_t s) {
  if (p.m <= 0) return hipSuccess;
  const dim3 grid(blocks_for(p.m, kSymWaves));
  if (fill)
    hipLaunchKernelGGL(k_c_two_level<true>, grid, dim3(kSymBlock), 0, s, p, pt_ptr, pt_row, cnt, flag, ovf, novf,
                       C_rowptr, C_col);
  else
    hipLaunchKernelGGL(k_c_two_level<false>, grid, dim3(kSymBlock), 0, s, p, pt_ptr, pt_row, cnt, flag, ovf,
                       novf, C_rowptr, C_col);
  return hipGetLastError();
}

// Bound on |C(i,:)| for the listed rows: min(m, sum of |R_I| over I with P(I,i) stored).
__global__ void k_c_bound_list(const int* __restrict__ pt_ptr, const int* __restrict__ pt_row,
                               const int* __restrict__ r, const int* __restrict__ list, int count, int m,
                               long long* bound) {
  const long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  if (k >= count) return;
  const int i = list[k];
  long long s = 0;
  for (int t = pt_ptr[i]; t < pt_ptr[i + 1]; ++t) s += r[pt_row[t]];
  bound[i] = s < m ? s : m;
}

hipError_t launch_c_bound_list(const int* pt_ptr, const int* pt_row, const int* r, const int* list, int count,
                               int m, long long* bound, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_c_bound_list, dim3(blocks_for(count, kSymBlock)), dim3(kSymBlock), 0, s, pt_ptr, pt_row,
                     r, list, count, m, bound);
  return hipGetLastError();
}

// =============================================================================================
// Owner tiles: slot[i] = (tile << kTileRowBits) | position of row i in its tile.
// =============================================================================================
__global__ void k_tile_slot(const int* __restrict__ tptr, const int* __restrict__ trows, int* slot) {
  const int t = blockIdx.x;
  const int b = tptr[t], e = tptr[t + 1];
  for (int q = b + threadIdx.x; q < e; q += kSymBlock) slot[trows[q]] = (t << kTileRowBits) | (q - b);
}

hipError_t launch_tile_slot(const int* tptr, const int* trows, int ntiles, int* slot, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_slot, dim3(ntiles), dim3(kSymBlock), 0, s, tptr, trows, slot);
  return hipGetLastError();
}

// =============================================================================================
// Launch-class codes of the row-form kernels (two-step products, atomic fold).  The short-row
// kernels take rows with at most kRowMulMaxLen keys; their lists are codes kCodeShort0 (the row
// of X has at most kHalfLanes entries) and kCodeShort1 (longer); other rows get the capacity
// code of their key bound.
//   mode 0 (rows of AP, two-step):   keys |R_I| = r[I], X row = A(I,:)
//   mode 1 (rows of C, two-step):    keys |C(i,:)|, X row = column i of P (pt_ptr)
//   mode 2 (fine rows, atomic fold): keys |R_I|; short only if P(I,:) and every row of C under
//                                    it have at most kRowMulMaxLen entries; rows with an empty
//                                    P(I,:) or R_I are dropped
// `short_ok` = 0 turns the short lists off.
// =============================================================================================
__global__ void k_rowform_codes(int mode, int nrows, const int* __restrict__ r, const int* __restrict__ x_ptr,
                                const int* __restrict__ c_ptr, const int* __restrict__ P_rowptr,
                                const int* __restrict__ P_col, int short_ok, int* code) {
  const long long k = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  if (k >= nrows) return;
  const int row = (int)k;
  long long keys;
  if (mode == 1)
    keys = c_ptr[row + 1] - c_ptr[row];
  else
    keys = r[row];
  int out = keys <= 0 ? -1 : dev_cap_log2(keys);
  if (mode == 2 && P_rowptr[row + 1] == P_rowptr[row]) out = -1;
  if (out >= 0 && short_ok && keys <= kRowMulMaxLen) {
    bool fits = true;
    if (mode == 2) {
      const int pb = P_rowptr[row], pe = P_rowptr[row + 1];
      fits = pe - pb <= kRowMulMaxLen;
      for (int e = pb; fits && e < pe; ++e) fits = c_ptr[P_col[e] + 1] - c_ptr[P_col[e]] <= kRowMulMaxLen;
    }
    if (fits) out = x_ptr[row + 1] - x_ptr[row] > kHalfLanes ? kCodeShort1 : kCodeShort0;
  }
  code[k] = out;
}

hipError_t launch_rowform_codes(int mode, int nrows, const int* r, const int* x_ptr, const int* c_ptr,
                                const int* P_rowptr, const int* P_col, bool short_ok, int* code, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowform_codes, dim3(blocks_for(nrows, kSymBlock)), dim3(kSymBlock), 0, s, mode, nrows, r,
                     x_ptr, c_ptr, P_rowptr, P_col, short_ok ? 1 : 0, code);
  return hipGetLastError();
}

}  // namespace ptapk
