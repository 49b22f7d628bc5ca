// Host-side logic of the symbolic phase that needs no GPU: hash-table capacities, the owner tiles
// and the hash multiplier of the short-row owner kernel.  Plain C++17: the library's host code
// includes it, and so does a CPU test that checks these functions without a GPU.
#pragma once

#include <algorithm>
#include <exception>
#include <functional>
#include <thread>
#include <vector>

#if defined(__HIPCC__)
#define PTAP_HD __host__ __device__
#else
#define PTAP_HD
#endif

namespace ptapk {
namespace host {

// LDS layout of the general owner kernel (one workgroup of `waves` wavefronts): the tile's values
// (TE doubles) and columns (TE ints), its row offsets (1025 ints), one wavefront scratch of
// `ws_bytes` bytes per wavefront (it holds doubles), then, for tables in LDS, `cap` doubles and
// `cap` ints per wavefront.  Every region starts on a 16-byte boundary: with the regions packed
// back to back, an odd TE left the doubles after the tile at addresses 4 mod 8, which FP64 LDS
// accesses do not support.  A null tile (tile in device memory) takes no room.
struct OwnerLayout {
  size_t tv, tc, trp, ws, vals, keys, total;
};
PTAP_HD inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
PTAP_HD inline OwnerLayout owner_general_layout(long long TE, long long cap, int waves, size_t ws_bytes,
                                                bool tile_in_lds, bool tables_in_lds) {
  OwnerLayout l{};
  size_t o = 0;
  if (tile_in_lds) {
    l.tv = o;
    o = align16(o + (size_t)TE * 8);
    l.tc = o;
    o = align16(o + (size_t)TE * 4);
    l.trp = o;
    o = align16(o + (size_t)1025 * 4);
  }
  l.ws = o;
  o = align16(o + (size_t)waves * ws_bytes);
  if (tables_in_lds) {
    l.vals = o;
    o = align16(o + (size_t)waves * (size_t)cap * 8);
    l.keys = o;
    o = align16(o + (size_t)waves * (size_t)cap * 4);
  }
  l.total = o;
  return l;
}

// Choice of the fold for PTAP_FOLD_AUTO.  Which of the two ways of adding P(I,:) (x) R_I into C
// is cheaper depends on the problem (Section 3 leaves the choice between the loops of Alg. 8 and
// Alg. 10 open): the owner fold forms some rows R_I more than once (a fine row whose entries of P
// fall in several tiles is formed in each) but adds in on-chip memory, the atomic fold forms each
// row once and adds every term with a device-wide FP64 atomic.  The estimates are linear in the
// symbolic phase's counts, with constants fitted (non-negative least squares on relative error)
// to the measured numeric times of both folds on one MI355X over seven workloads: 27-point
// lognormal operators at 128^3 and 64^3 and a 7-point one at 128^3 with trilinear P, smoothed
// aggregation with one and two Jacobi steps at 96^3 and two at 48^3, and a 4x4-block operator.
//   owner  = 0.161 ms per million rows formed + 0.00334 ms per million products formed
//            (products of the needed rows times rows formed / rows needed)
//   atomic = 0.100 ms per million rows formed + 0.0206 ms per million fold terms
// (the atomic fold forms each needed row once per pass).  The fit picks the faster fold on all
// seven; the terms it drops (the owner fold's own adds, the atomic fold's products) came out at
// zero weight.
struct FoldEstimate {
  double owner_ms, atomic_ms;
};
inline FoldEstimate fold_estimate(long long rows_needed, long long rows_formed_owner, long long products,
                                  long long fold_terms, bool two_passes) {
  FoldEstimate e{0.0, 0.0};
  if (rows_needed <= 0) return e;
  const double r = (double)rows_formed_owner / (double)rows_needed;
  e.owner_ms = 0.161e-6 * (double)rows_formed_owner + 0.00334e-6 * (double)products * r;
  e.atomic_ms = 0.100e-6 * (double)rows_needed * (two_passes ? 2.0 : 1.0) + 0.0206e-6 * (double)fold_terms;
  return e;
}

inline int next_pow2(long long v) {
  long long c = 1;
  while (c < v) c <<= 1;
  return (int)std::min<long long>(c, 1LL << 30);
}

// Table capacity for a row whose key set has at most `need` distinct keys: a power of two of at
// least 2*need slots (load factor <= 1/2), never below one slot per lane.
inline int cap_for(long long need) { return std::max(64, next_pow2(2 * std::max(need, 1LL))); }

// log2 of cap_for(need) for need >= 1: the smallest power of two >= 2*need, at least 64 and at
// most 2^30.
inline int cap_log2(long long need) {
  const unsigned long long v = 2ULL * (unsigned long long)need;
  const int b = v <= 64 ? 6 : 64 - __builtin_clzll(v - 1);
  return std::min(b, 30);
}

// Tiles of rows of C for the owner fold, grown breadth-first over the graph of C's pattern (row
// r is adjacent to the columns of row r): starting from the lowest unassigned row of the range
// [lo, hi), rows of that range are taken in BFS order while the tile holds at most TE entries and
// TR rows.  On meshes this gives compact tiles, so fewer fine rows touch two tiles than with
// contiguous ranges of rows.  A row longer than TE forms a tile of its own (tglob = 1: kept in
// device memory).  Rows within a tile are listed in ascending order.  Only state[lo..hi) is read
// or written, so ranges can be grown at the same time.
inline void grow_range(int lo, int hi, const int* cptr, const int* ccol, int TE, int TR, int* state,
                       std::vector<int>& tptr, std::vector<int>& trows, std::vector<char>& tglob) {
  // state: -1 free, -2 queued for the tile being grown, >= 0 taken
  std::vector<int> queue;
  queue.reserve(4096);
  tptr.assign(1, 0);
  trows.clear();
  tglob.clear();
  const unsigned span = (unsigned)(hi - lo);
  int taken = 0;
  for (int seed = lo; seed < hi; ++seed) {
    if (state[seed] != -1) continue;
    const int T = (int)tglob.size();
    if (cptr[seed + 1] - cptr[seed] > TE) {
      state[seed] = T;
      tptr.push_back(++taken);
      tglob.push_back(1);
      continue;
    }
    queue.clear();
    queue.push_back(seed);
    state[seed] = -2;
    size_t head = 0;
    long long acc = 0;
    int nrows = 0;
    // entries and rows queued beyond `head`: once taking every queued row would pass a limit,
    // the tile is sure to stop within the queue, so rows taken from then on need not queue
    // their neighbours (the tile comes out the same)
    long long queued = cptr[seed + 1] - cptr[seed];
    while (head < queue.size()) {
      const int r = queue[head];
      const int sz = cptr[r + 1] - cptr[r];
      if (acc + sz > TE || nrows >= TR) break;
      ++head;
      acc += sz;
      queued -= sz;
      ++nrows;
      state[r] = T;
      if (acc + queued > TE || nrows + (long long)(queue.size() - head) > TR) continue;
      for (int k = cptr[r]; k < cptr[r + 1]; ++k) {
        const int c = ccol[k];
        if ((unsigned)(c - lo) < span && state[c] == -1) {
          state[c] = -2;
          queue.push_back(c);
          queued += cptr[c + 1] - cptr[c];
        }
      }
    }
    for (size_t q = head; q < queue.size(); ++q) state[queue[q]] = -1;  // not taken
    taken += nrows;
    tptr.push_back(taken);
    tglob.push_back(0);
  }
  // list each tile's rows in ascending order: one pass over the range puts every row at the next
  // free position of its tile
  trows.resize((size_t)taken);
  std::vector<int> pos(tptr.begin(), tptr.end() - 1);
  for (int i = lo; i < hi; ++i) trows[pos[state[i]]++] = i;
}

// Multiplier of the short-row owner kernel's R_I hash (slot = top 6 bits of key * mul, linear
// probing over 64 slots).  The golden-ratio multiplier crowds the keys of some mesh sizes onto few
// slots (a stencil row's keys are i + dx + dy s + dz s^2 for the grid side s), so candidates are
// scored on a fixed sample of C's rows, which stand in for the rows R_I (both are sets of nearby
// coarse columns): a row's columns inserted into an empty table, then the columns of the row of
// its first column looked up, as the fold looks the columns of C's rows up in R_I.  The golden
// ratio stays unless it needs more than 1.3 times the probes of the best candidate: it spreads
// nearby keys evenly, which the probe count does not credit (simultaneous table accesses of a
// half-wavefront meet less often), and measured at 128^3 a candidate with 8% fewer probes ran 9%
// slower.  Candidates and sample are fixed (the candidates come from splitmix64 with a fixed
// seed), so a plan gets the same multiplier on every machine.
inline unsigned choose_hash_mul(int m, const int* cptr, const int* ccol) {
  constexpr int kCands = 16, kSample = 512, kSlots = 64, kShift = 26, kMaxKeys = 32;
  unsigned cand[kCands];
  cand[0] = 0x9E3779B1u;
  unsigned long long z = 0x243F6A8885A308D3ULL;
  for (int c = 1; c < kCands; ++c) {
    z += 0x9E3779B97F4A7C15ULL;
    unsigned long long x = z;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    x ^= x >> 31;
    cand[c] = (unsigned)(x >> 32) | 1u;
  }
  const int S = std::min(m, kSample);
  int keys[kSlots];
  // probes to find `key` (or its empty slot, where an insert stores it)
  auto probe = [&](int key, unsigned mul, bool insert) {
    unsigned sl = ((unsigned)key * mul) >> kShift;
    long long n = 1;
    while (keys[sl] != -1 && keys[sl] != key) {
      sl = (sl + 1) & (kSlots - 1);
      ++n;
    }
    if (insert) keys[sl] = key;
    return n;
  };
  long long best = -1, golden = 0;
  unsigned pick = cand[0];
  for (int c = 0; c < kCands; ++c) {
    long long probes = 0;
    for (int k = 0; k < S; ++k) {
      const int r = (int)((long long)k * m / S);
      const int b = cptr[r], e = cptr[r + 1];
      if (e == b || e - b > kMaxKeys) continue;
      std::fill(keys, keys + kSlots, -1);
      for (int q = b; q < e; ++q) probes += probe(ccol[q], cand[c], true);
      const int r2 = ccol[b];
      for (int q = cptr[r2]; q < cptr[r2 + 1]; ++q) probes += probe(ccol[q], cand[c], false);
    }
    if (c == 0) golden = probes;
    if (best < 0 || probes < best) {
      best = probes;
      pick = cand[c];
    }
  }
  return golden * 10 > best * 13 ? pick : cand[0];
}

// All rows of C in tiles: the rows are split into up to kGrowParts contiguous ranges of at least
// kGrowPartRows rows, grown on threads of their own, and the ranges' tiles listed in range order.
// The split depends on m only, so the tiles are the same on every machine.
constexpr int kGrowParts = 8;
constexpr int kGrowPartRows = 32768;

inline int grow_parts(int m) { return (int)std::max<long long>(1, std::min<long long>(kGrowParts, m / kGrowPartRows)); }

// Rows [lo, hi) of range p of grow_parts(m) ranges.
inline void grow_range_bounds(int m, int parts, int p, int& lo, int& hi) {
  lo = (int)((long long)m * p / parts);
  hi = (int)((long long)m * (p + 1) / parts);
}

// A range reads only its own rows of C (cptr[lo..hi] and their columns), so a caller that copies
// C's columns range by range passes wait_part(p), which returns once range p's columns are in
// place; row pointers must all be in place on entry.
inline void grow_tiles(int m, const int* cptr, const int* ccol, int TE, int TR, std::vector<int>& tptr,
                std::vector<int>& trows, std::vector<char>& tglob,
                const std::function<void(int)>& wait_part = std::function<void(int)>()) {
  const int parts = grow_parts(m);
  std::vector<int> state(m, -1);
  std::vector<std::vector<int>> pp(parts), pr(parts);
  std::vector<std::vector<char>> pg(parts);
  std::vector<std::exception_ptr> err(parts);
  auto work = [&](int p) {
    try {
      int lo, hi;
      grow_range_bounds(m, parts, p, lo, hi);
      if (wait_part) wait_part(p);
      grow_range(lo, hi, cptr, ccol, TE, TR, state.data(), pp[p], pr[p], pg[p]);
    } catch (...) {
      err[p] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  for (int p = 1; p < parts; ++p) {
    try {
      th.emplace_back(work, p);
    } catch (...) {
      work(p);  // no thread to spare: grow the range here
    }
  }
  work(0);
  for (std::thread& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  tptr.assign(1, 0);
  trows.clear();
  tglob.clear();
  for (int p = 0; p < parts; ++p) {
    const int base = (int)trows.size();
    for (size_t k = 1; k < pp[p].size(); ++k) tptr.push_back(base + pp[p][k]);
    trows.insert(trows.end(), pr[p].begin(), pr[p].end());
    tglob.insert(tglob.end(), pg[p].begin(), pg[p].end());
  }
}

}  // namespace host
}  // namespace ptapk
