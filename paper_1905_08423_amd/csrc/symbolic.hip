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
// Inserting keys into a wavefront's LDS hash tables.  Each lane takes its own segment of `col`
// ([s, s + l)), eight loads at a time; every round inserts at most one key per lane, and after a
// round each table's count of keys grows by the new keys of the lanes that share it (`group`
// masks them).  A table that passes `limit` keys stops taking keys (*ovf), so with limit + the
// lanes of its group below its capacity, probing always finds a free slot.
// =============================================================================================
template <class Ins>
__device__ __forceinline__ void insert_segments(int s, int l, const int* __restrict__ col,
                                                unsigned long long group, int limit, int& occ, bool& ovf,
                                                Ins&& ins) {
  const int maxl = wave_max(l);
  for (int e0 = 0; e0 < maxl; e0 += 8) {
    int key[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) key[j] = e0 + j < l ? col[s + e0 + j] : -1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool fresh = key[j] >= 0 && !ovf && ins(key[j]);
      occ += __popcll(ballot(fresh) & group);
      ovf = ovf || occ > limit;
    }
  }
}

// The same for the rows of P whose extents a table's L lanes left in ext[0..L) (start, length;
// (0, 0) for none): eight lanes take one row, so a load instruction reads L/8 runs of
// consecutive entries instead of one scattered entry per lane (in the |R_I| pass 12% faster;
// the C pass, whose lists of rows are longer, ran 12% slower with it).  In round u the lanes of group g
// take row u * (L/8) + g; rounds repeat for entries beyond the first eight (maxl: the longest
// row over the wavefront).
template <int L, class Ins>
__device__ __forceinline__ void insert_rows_grouped(const int2* ext, int maxl, const int* __restrict__ col,
                                                    unsigned long long group, int limit, int& occ, bool& ovf,
                                                    Ins&& ins) {
  constexpr int G = 8, PER = L / G;
  const int bl = lane() % L, g = bl / G, t = bl % G;
  for (int e0 = 0; e0 < maxl; e0 += G) {
    int key[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int2 ex = ext[u * PER + g];
      key[u] = e0 + t < ex.y ? col[ex.x + e0 + t] : -1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool fresh = key[u] >= 0 && !ovf && ins(key[u]);
      occ += __popcll(ballot(fresh) & group);
      ovf = ovf || occ > limit;
    }
  }
}

// =============================================================================================
// |R_I| and w_I in one pass (Alg. 1 / Alg. 2): each half-wavefront forms the key set of one row
// I of AP in a 64-slot LDS table, its lanes taking the entries J of A(I,:) and inserting the
// columns of P(J,:).  A row with more than kApMaxKeys keys is listed in `ovf` instead (its |R_I|
// comes from the launches by capacity class).  w[I] = min(w_I, m), w_I = sum of nnz(P(J,:)).
// =============================================================================================
constexpr int kApCap = 64;
constexpr int kApMaxKeys = kApCap - 32 - 1;

__global__ __launch_bounds__(kSymBlock) void k_ap_count(Patterns p, int* r, int* w, int* ovf, int* novf) {
  __shared__ int keys_all[2 * kSymWaves][kApCap];
  __shared__ int2 ext_all[2 * kSymWaves][32];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int h = ln >> 5, sub = ln & 31;
  const long long I64 = ((long long)blockIdx.x * kSymWaves + wid) * 2 + h;
  if (((long long)blockIdx.x * kSymWaves + wid) * 2 >= p.n) return;  // uniform over the wavefront
  const bool live = I64 < p.n;
  const int I = live ? (int)I64 : 0;
  int* keys = keys_all[2 * wid + h];
  keys[sub] = EMPTY;
  keys[sub + 32] = EMPTY;
  wave_sync();
  const unsigned long long group = h ? 0xFFFFFFFF00000000ULL : 0x00000000FFFFFFFFULL;
  const int a0 = live ? p.A_rowptr[I] : 0, la = live ? p.A_rowptr[I + 1] - a0 : 0;
  const int maxa = wave_max(la);
  long long prod = 0;
  int occ = 0;
  bool over = false;
  int2* ext = ext_all[2 * wid + h];
  for (int eb = 0; eb < maxa; eb += 32) {
    int s = 0, l = 0;
    if (eb + sub < la) {
      const int J = p.A_col[a0 + eb + sub];
      s = p.P_rowptr[J];
      l = p.P_rowptr[J + 1] - s;
    }
    prod += l;
    ext[sub] = make_int2(s, l);
    wave_sync();
    insert_rows_grouped<32>(ext, wave_max(l), p.P_col, group, kApMaxKeys, occ, over, [&](int key) {
      bool fresh;
      hs_insert<false>(keys, kApCap - 1, 32 - 6, key, fresh);
      return fresh;
    });
    wave_sync();
  }
#pragma unroll
  for (int d = 16; d > 0; d >>= 1) prod += __shfl_xor(prod, d, WAVE);  // within the half
  if (live && sub == 0) {
    w[I] = (int)(prod < p.m ? prod : p.m);
    r[I] = over ? 0 : occ;
    if (over) ovf[atomicAdd(novf, 1)] = I;
  }
}

hipError_t launch_ap_count(const Patterns& p, int* r, int* w, int* ovf, int* novf, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ap_count, dim3(blocks_for(p.n, 2 * kSymWaves)), dim3(kSymBlock), 0, s, p, r, w, ovf, novf);
  return hipGetLastError();
}

// =============================================================================================
// Pattern of C by a two-level union (Eq. allatoncerow): C(i,:) is the union over I with P(I,i)
// stored of the union over J in A(I,:) of P(J,:), so with S_i the set of all such J,
// C(i,:) = union over J in S_i of P(J,:).  One wavefront per row i builds S_i in an LDS table
// (each half-wavefront takes one I at a time, its lanes the entries of A(I,:)), then C(i,:) in a
// second table (each lane one J of S_i): neighbouring fine rows I share most of their J, so each
// distinct J is walked once instead of once per I.  A row whose S_i or C(i,:) outgrows its table
// is flagged and listed in `ovf` (count pass) and left to the launches by capacity class.
// Count pass: cnt[i] = |C(i,:)|; a row of at most kRowStore columns goes, sorted, to its slot of
// the row store (if one is given) and is copied into C_col once the row pointers are known, so
// that only longer rows take the fill pass.  flag[i]: 0 fill pass, 1 class launches, 2 row
// store; *nfill counts the rows of flag 0.  Fill pass: the sorted columns at C_rowptr[i], for
// rows of flag 0.
// =============================================================================================
constexpr int kTwoSCap = 512, kTwoSMax = kTwoSCap - WAVE - 1;
constexpr int kTwoCCap = 256, kTwoCMax = kTwoCCap - WAVE - 1;

struct TwoLevelScratch {
  int skeys[kTwoSCap];
  int slist[kTwoSMax + 1];
  int ckeys[kTwoCCap];
  int clist[kTwoCMax + 1];
};

template <bool FILL>
__global__ __launch_bounds__(kSymBlock) void k_c_two_level(Patterns p, const int* __restrict__ pt_ptr,
                                                           const int* __restrict__ pt_row, int* cnt,
                                                           unsigned char* flag, int* ovf, int* novf,
                                                           const int* __restrict__ C_rowptr, int* C_col,
                                                           int* store, int* nfill, int row0, int row1) {
  __shared__ TwoLevelScratch scr[kSymWaves];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int h = ln >> 5, sub = ln & 31;
  const long long i64 = row0 + (long long)blockIdx.x * kSymWaves + wid;
  if (i64 >= row1) return;  // uniform over the wavefront
  const int i = (int)i64;
  if (FILL && flag[i] != 0) return;
  TwoLevelScratch& sc = scr[wid];
  for (int q = ln; q < kTwoSCap; q += WAVE) sc.skeys[q] = EMPTY;
  for (int q = ln; q < kTwoCCap; q += WAVE) sc.ckeys[q] = EMPTY;
  wave_sync();
  constexpr int sshift = 32 - 9, cshift = 32 - 8;
  static_assert(kTwoSCap == 512 && kTwoCCap == 256, "shifts assume these capacities");
  auto s_ins = [&](int key) {
    bool fresh;
    hs_insert<false>(sc.skeys, kTwoSCap - 1, sshift, key, fresh);
    return fresh;
  };
  auto c_ins = [&](int key) {
    bool fresh;
    hs_insert<false>(sc.ckeys, kTwoCCap - 1, cshift, key, fresh);
    return fresh;
  };
  // level 1: S_i from the rows of A under the fine rows I of column i of P, 64 of them at a time
  const int t0 = pt_ptr[i], nI = pt_ptr[i + 1] - t0;
  int ns = 0;
  bool over = false;
  for (int xb = 0; xb < nI; xb += WAVE) {
    const int nb = min(WAVE, nI - xb);
    int a0 = 0, al = 0;
    if (ln < nb) {
      const int I = pt_row[t0 + xb + ln];
      a0 = p.A_rowptr[I];
      al = p.A_rowptr[I + 1] - a0;
    }
    const int maxal = wave_max(al);
    for (int x = 0; x < nb; x += 4) {  // two rows I per half-wavefront per round
      const int xa = x + h, xc = x + 2 + h;
      // (every lane takes part in the shuffles; the lengths of rows past the batch are zeroed after)
      const int sa = __shfl(a0, xa & (WAVE - 1), WAVE), la_raw = __shfl(al, xa & (WAVE - 1), WAVE);
      const int sb = __shfl(a0, xc & (WAVE - 1), WAVE), lb_raw = __shfl(al, xc & (WAVE - 1), WAVE);
      const int la_ = xa < nb ? la_raw : 0, lb = xc < nb ? lb_raw : 0;
      for (int e0 = 0; e0 < maxal; e0 += 32) {
        const int ka = e0 + sub < la_ ? p.A_col[sa + e0 + sub] : -1;
        const int kb = e0 + sub < lb ? p.A_col[sb + e0 + sub] : -1;
        bool fresh = ka >= 0 && !over && s_ins(ka);
        ns += __popcll(ballot(fresh));
        over = over || ns > kTwoSMax;
        fresh = kb >= 0 && !over && s_ins(kb);
        ns += __popcll(ballot(fresh));
        over = over || ns > kTwoSMax;
      }
    }
  }
  int nc = 0;
  if (!over) {
    // S_i as a list
    int base = 0;
    for (int s0 = 0; s0 < kTwoSCap; s0 += WAVE) {
      const int k = sc.skeys[s0 + ln];
      const unsigned long long mk = ballot(k != EMPTY);
      if (k != EMPTY) sc.slist[base + prefix_count(mk)] = k;
      base += __popcll(mk);
    }
    wave_sync();
    // level 2: C(i,:) from the rows of P under S_i, one J per lane
    for (int xb = 0; xb < ns && !over; xb += WAVE) {
      int s = 0, l = 0;
      if (xb + ln < ns) {
        const int J = sc.slist[xb + ln];
        s = p.P_rowptr[J];
        l = p.P_rowptr[J + 1] - s;
      }
      insert_segments(s, l, p.P_col, ~0ULL, kTwoCMax, nc, over, c_ins);
    }
  }
  // C(i,:)'s columns in ascending order at out
  auto emit = [&](int* out) {
    int base = 0;
    for (int s0 = 0; s0 < kTwoCCap; s0 += WAVE) {
      const int k = sc.ckeys[s0 + ln];
      const unsigned long long mk = ballot(k != EMPTY);
      if (k != EMPTY) sc.clist[base + prefix_count(mk)] = k;
      base += __popcll(mk);
    }
    wave_sync();
    for (int x = ln; x < base; x += WAVE) {
      const int key = sc.clist[x];
      int rank = 0;
      for (int y = 0; y < base; ++y) rank += sc.clist[y] < key;
      out[rank] = key;
    }
  };
  if constexpr (!FILL) {
    const bool stored = !over && store && nc <= kRowStore;
    if (stored) emit(store + (size_t)i * kRowStore);
    if (ln == 0) {
      cnt[i] = over ? 0 : nc;
      flag[i] = over ? 1 : (stored ? 2 : 0);
      if (over) ovf[atomicAdd(novf, 1)] = i;
      if (!over && !stored) atomicAdd(nfill, 1);
    }
  } else {
    if (over) return;  // not reached for rows the count pass kept
    emit(C_col + C_rowptr[i]);
  }
}

// Rows the count pass kept in the row store, copied to their place in C_col: one thread per
// (row, position), so reads and writes run along the rows.
__global__ __launch_bounds__(kSymBlock) void k_c_from_store(const int* __restrict__ C_rowptr,
                                                            const int* __restrict__ store,
                                                            const unsigned char* __restrict__ flag, int row0,
                                                            int row1, int* C_col) {
  const long long t = (long long)blockIdx.x * kSymBlock + threadIdx.x;
  const long long i = row0 + t / kRowStore;
  const int e = (int)(t % kRowStore);
  if (i >= row1 || flag[i] != 2) return;
  const int b = C_rowptr[i];
  if (e < C_rowptr[i + 1] - b) C_col[b + e] = store[(size_t)i * kRowStore + e];
}

hipError_t launch_c_from_store(const int* C_rowptr, const int* store, const unsigned char* flag, int row0, int row1,
                               int* C_col, hipStream_t s) {
  if (row1 <= row0) return hipSuccess;
  hipLaunchKernelGGL(k_c_from_store, dim3(blocks_for(((long long)row1 - row0) * kRowStore, kSymBlock)),
                     dim3(kSymBlock), 0, s, C_rowptr, store, flag, row0, row1, C_col);
  return hipGetLastError();
}

hipError_t launch_c_two_level(const Patterns& p, const int* pt_ptr, const int* pt_row, bool fill, int* cnt,
                              unsigned char* flag, int* ovf, int* novf, const int* C_rowptr, int* C_col,
                              int* store, int* nfill, int row0, int row1, hipStream_t s) {
  if (row0 < 0 || row1 > p.m) return hipErrorInvalidValue;
  if (row1 <= row0) return hipSuccess;
  const dim3 grid(blocks_for((long long)row1 - row0, kSymWaves));
  if (fill)
    hipLaunchKernelGGL(k_c_two_level<true>, grid, dim3(kSymBlock), 0, s, p, pt_ptr, pt_row, cnt, flag, ovf, novf,
                       C_rowptr, C_col, store, nfill, row0, row1);
  else
    hipLaunchKernelGGL(k_c_two_level<false>, grid, dim3(kSymBlock), 0, s, p, pt_ptr, pt_row, cnt, flag, ovf,
                       novf, C_rowptr, C_col, store, nfill, row0, row1);
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

// =============================================================================================
// Launch classes of the adjoint (dA = P dC P^T and dP = A P dC^T + A^T P dC, Section 3's products
// read backwards): the table of fine row I holds U_I, the distinct columns of the rows of dC
// (C's pattern) under P(I,:), which include R_I's.  Each half-wavefront counts U_I for one row in
// a 128-slot LDS table, its lanes taking the entries of P(I,:); a row with more than
// kAdjCountMax distinct columns takes min(walk, m) as its bound instead, walk being the number of
// entries of those rows of C.  need = max(|U_I| or the bound, |R_I|, 1); rows whose P(I,:) has at
// most kAdjMaxSegs entries, whose walk is at most kAdjMaxWalk and whose table fits `fast_cap`
// slots get code 32 + log2(capacity) (the short-row kernel), the others log2(capacity); rows
// with an empty P(I,:) get -1.
// =============================================================================================
constexpr int kAdjCountCap = 128;
constexpr int kAdjCountMax = kAdjCountCap - 32 - 1;

__global__ __launch_bounds__(kSymBlock) void k_adj_codes(Patterns p, const int* __restrict__ r,
                                                         const int* __restrict__ C_rowptr,
                                                         const int* __restrict__ C_col, int fast_cap, int* code) {
  __shared__ int keys_all[2 * kSymWaves][kAdjCountCap];
  const int wid = threadIdx.x / WAVE, ln = lane();
  const int h = ln >> 5, sub = ln & 31;
  const long long first = ((long long)blockIdx.x * kSymWaves + wid) * 2;
  if (first >= p.n) return;  // uniform over the wavefront
  const long long I64 = first + h;
  const bool live = I64 < p.n;
  const int I = live ? (int)I64 : 0;
  int* keys = keys_all[2 * wid + h];
  for (int q = sub; q < kAdjCountCap; q += 32) keys[q] = EMPTY;
  wave_sync();
  const unsigned long long group = h ? 0xFFFFFFFF00000000ULL : 0x00000000FFFFFFFFULL;
  const int p0 = live ? p.P_rowptr[I] : 0, np = live ? p.P_rowptr[I + 1] - p0 : 0;
  const int maxp = wave_max(np);
  long long walk = 0;
  int occ = 0;
  bool over = false;
  for (int eb = 0; eb < maxp; eb += 32) {
    int s = 0, l = 0;
    if (eb + sub < np) {
      const int i = p.P_col[p0 + eb + sub];
      s = C_rowptr[i];
      l = C_rowptr[i + 1] - s;
    }
    walk += l;
    insert_segments(s, l, C_col, group, kAdjCountMax, occ, over, [&](int key) {
      bool fresh;
      hs_insert<false>(keys, kAdjCountCap - 1, 32 - 7, key, fresh);
      return fresh;
    });
  }
#pragma unroll
  for (int d = 16; d > 0; d >>= 1) walk += __shfl_xor(walk, d, WAVE);  // within the half
  if (live && sub == 0) {
    int out = -1;
    if (np > 0) {
      long long need = over ? (walk < p.m ? walk : p.m) : occ;
      need = need > r[I] ? need : r[I];
      need = need > 1 ? need : 1;
      const int b = dev_cap_log2(need);
      const bool fast = np <= kAdjMaxSegs && walk <= kAdjMaxWalk && (1LL << b) <= fast_cap;
      out = fast ? 32 + b : b;
    }
    code[I] = out;
  }
}

hipError_t launch_adj_codes(const Patterns& p, const int* r, const int* C_rowptr, const int* C_col, int fast_cap,
                            int* code, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_codes, dim3(blocks_for(p.n, 2 * kSymWaves)), dim3(kSymBlock), 0, s, p, r, C_rowptr, C_col,
                     fast_cap, code);
  return hipGetLastError();
}

// =============================================================================================
// Bounds that fix the owner tiles' size before |R_I| is known: out[0] = max over fine rows I with
// a non-empty P(I,:) of min over i in P(I,:) of |C(i,:)| (R_I lies within every such C(i,:), so
// this bounds |R_I| for every row the fold needs); out[1] = max over I of max(nnz(P(I,:)),
// nnz(A(I,:))).  out zeroed by the caller.
// =============================================================================================
__global__ __launch_bounds__(kSymBlock) void k_row_bounds(Patterns p, const int* __restrict__ C_rowptr,
                                                          unsigned* out) {
  __shared__ int red[2][kSymWaves];
  int rb = 0, lm = 0;
  for (long long I = (long long)blockIdx.x * kSymBlock + threadIdx.x; I < p.n; I += (long long)gridDim.x * kSymBlock) {
    const int pb = p.P_rowptr[I], pe = p.P_rowptr[I + 1];
    if (pe > pb) {
      int mn = INT32_MAX;
      for (int e = pb; e < pe; ++e) {
        const int i = p.P_col[e];
        mn = min(mn, C_rowptr[i + 1] - C_rowptr[i]);
      }
      rb = max(rb, mn);
    }
    lm = max(lm, max(pe - pb, p.A_rowptr[I + 1] - p.A_rowptr[I]));
  }
  rb = wave_max(rb);
  lm = wave_max(lm);
  const int wid = threadIdx.x / WAVE;
  if (lane() == 0) {
    red[0][wid] = rb;
    red[1][wid] = lm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSymWaves; ++w) {
      rb = max(rb, red[0][w]);
      lm = max(lm, red[1][w]);
    }
    atomicMax(out, (unsigned)rb);
    atomicMax(out + 1, (unsigned)lm);
  }
}

hipError_t launch_row_bounds(const Patterns& p, const int* C_rowptr, unsigned* out, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_bounds, dim3(std::min(blocks_for(p.n, kSymBlock), 1024)), dim3(kSymBlock), 0, s, p,
                     C_rowptr, out);
  return hipGetLastError();
}

}  // namespace ptapk
