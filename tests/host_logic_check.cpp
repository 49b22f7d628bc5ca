// CPU checks of the symbolic phase's host logic (hash-table capacities, owner tiles, the hash
// multiplier of the short-row owner kernel), built with g++ by tests/test_host_logic.py.  Prints
// one "ok <check>" line per check and exits non-zero at the first failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1905_08423_amd/csrc/host_logic.hpp"

using namespace ptapk::host;

static void fail(const char* what, long long a = 0, long long b = 0) {
  std::printf("FAIL %s %lld %lld\n", what, a, b);
  std::exit(1);
}

// Pattern of the 27-point stencil on an s^3 grid (rows sorted ascending).
static void stencil27(int s, std::vector<int>& ptr, std::vector<int>& col) {
  const int m = s * s * s;
  ptr.assign(m + 1, 0);
  col.clear();
  col.reserve((size_t)m * 27);
  for (int z = 0; z < s; ++z)
    for (int y = 0; y < s; ++y)
      for (int x = 0; x < s; ++x) {
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int X = x + dx, Y = y + dy, Z = z + dz;
              if (X < 0 || Y < 0 || Z < 0 || X >= s || Y >= s || Z >= s) continue;
              col.push_back((Z * s + Y) * s + X);
            }
        ptr[(z * s + y) * s + x + 1] = (int)col.size();
      }
}

// Every row in exactly one tile; rows ascending within a tile; a tile holds at most TE entries
// and TR rows, or is one row longer than TE marked as kept in device memory; no tile crosses a
// boundary of the contiguous row ranges the rows are split into; the same tiles a second time.
static void check_tiles(const char* name, int m, const std::vector<int>& ptr,
                        const std::vector<int>& col, int TE, int TR) {
  std::vector<int> tptr, trows, tptr2, trows2;
  std::vector<char> tglob, tglob2;
  grow_tiles(m, ptr.data(), col.data(), TE, TR, tptr, trows, tglob);
  grow_tiles(m, ptr.data(), col.data(), TE, TR, tptr2, trows2, tglob2);
  if (tptr != tptr2 || trows != trows2 || tglob != tglob2) fail("tiles not deterministic");
  const int T = (int)tglob.size();
  if ((int)tptr.size() != T + 1 || tptr[0] != 0 || tptr[T] != m || (int)trows.size() != m)
    fail("tile lists do not cover the rows", tptr.back(), m);
  const int parts = (int)std::max<long long>(1, std::min<long long>(kGrowParts, m / kGrowPartRows));
  auto range_of = [&](int r) {
    int p = (int)((long long)r * parts / m);
    while (p + 1 < parts && (long long)m * (p + 1) / parts <= r) ++p;
    while (p > 0 && (long long)m * p / parts > r) --p;
    return p;
  };
  std::vector<int> seen(m, 0);
  for (int t = 0; t < T; ++t) {
    const int a = tptr[t], b = tptr[t + 1];
    if (b <= a) fail("empty tile", t);
    long long entries = 0;
    for (int q = a; q < b; ++q) {
      const int r = trows[q];
      if (r < 0 || r >= m) fail("row out of range", r);
      if (seen[r]++) fail("row in two tiles", r);
      if (q > a && trows[q - 1] >= r) fail("rows not ascending in a tile", t);
      if (range_of(r) != range_of(trows[a])) fail("tile crosses a row range", t, r);
      entries += ptr[r + 1] - ptr[r];
    }
    if (tglob[t]) {
      if (b - a != 1 || entries <= TE) fail("device-memory tile is not one long row", t);
    } else if (entries > TE || b - a > TR) {
      fail("tile over its limits", entries, b - a);
    }
  }
  std::printf("ok tiles %s (%d rows, %d ranges, %d tiles)\n", name, m, parts, T);
}


// LDS layout of the general owner kernel: every region aligned to 16 bytes and inside the total,
// regions in order without overlap, for every tile size up to 8192 entries and the table
// capacities the kernel takes.  The layout the kernel used before packed the regions back to back
// (tile values, columns, 1025 row offsets rounded to 16 bytes, then the wavefront scratch that
// holds doubles): for an odd tile size that put the doubles at addresses 4 mod 8.
static void check_owner_layout() {
  const size_t ws_bytes = 1024;  // WaveScratch: 64 ints, 64 ints, 64 doubles
  for (long long TE = 1; TE <= 8192; ++TE)
    for (long long cap : {64LL, 128LL, 256LL, 512LL, 1024LL})
      for (int waves : {4, 8})
        for (int tile = 0; tile < 2; ++tile)
          for (int tab = 0; tab < 2; ++tab) {
            const OwnerLayout l = owner_general_layout(TE, cap, waves, ws_bytes, tile, tab);
            size_t end = 0;
            auto region = [&](size_t off, size_t bytes, const char* what) {
              if (off % 16 != 0) fail(what, TE, (long long)off);
              if (off < end) fail("regions overlap", TE, (long long)off);
              end = off + bytes;
              if (end > l.total) fail("region past the total", TE, (long long)end);
            };
            if (tile) {
              region(l.tv, (size_t)TE * 8, "tile values misaligned");
              region(l.tc, (size_t)TE * 4, "tile columns misaligned");
              region(l.trp, 1025 * 4, "row offsets misaligned");
            }
            region(l.ws, (size_t)waves * ws_bytes, "wavefront scratch misaligned");
            if (tab) {
              region(l.vals, (size_t)waves * (size_t)cap * 8, "table values misaligned");
              region(l.keys, (size_t)waves * (size_t)cap * 4, "table keys misaligned");
            }
          }
  // the packed layout: scratch at 12 TE + 4112 bytes, 4 mod 8 for every odd TE
  for (long long TE = 1; TE < 5000; TE += 2)
    if ((12 * TE + 4112) % 8 != 4) fail("packed layout arithmetic", TE, 0);
  std::printf("ok owner layout aligned\n");
}


// The fold cost model: the measured cases of its fit each pick the fold that was faster.
static void check_fold_estimate() {
  struct Case {
    const char* name;
    long long needed, formed, products, fold;
    bool atomic_faster;
  } cases[] = {
      {"27pt 128^3 trilinear", 2097152, 2891040, 186169411, 86938307, false},
      {"SA one step 96^3", 884736, 1475244, 105154048, 40707584, false},
      {"SA two steps 96^3", 884736, 3173617, 284890312, 274625000, false},
      {"27pt 64^3 trilinear", 262144, 388764, 22665187, 10503459, false},
      {"7pt 128^3 trilinear", 2097152, 2891040, 48556211, 69839855, false},
      {"SA two steps 48^3", 110592, 604294, 33386248, 30959144, true},
      {"4x4 blocks 40^3", 256000, 838104, 474552000, 187149248, true},
  };
  for (const Case& c : cases) {
    const FoldEstimate e = fold_estimate(c.needed, c.formed, c.products, c.fold, false);
    if ((e.atomic_ms < e.owner_ms) != c.atomic_faster) fail(c.name, (long long)(e.owner_ms * 1e3), (long long)(e.atomic_ms * 1e3));
  }
  const FoldEstimate z = fold_estimate(0, 0, 0, 0, false);
  if (z.owner_ms != 0.0 || z.atomic_ms != 0.0) fail("empty problem", 0, 0);
  std::printf("ok fold estimate\n");
}

int main() {
  check_fold_estimate();
  check_owner_layout();
  // capacities: cap_log2 is the exponent of cap_for
  for (long long need = 1; need <= 300000; ++need)
    if ((1LL << cap_log2(need)) != cap_for(need)) fail("cap_log2", need);
  for (int e = 18; e <= 33; ++e)
    for (long long d = -2; d <= 2; ++d) {
      const long long need = (1LL << e) + d;
      if ((1LL << cap_log2(need)) != cap_for(need)) fail("cap_log2 large", need);
    }
  std::printf("ok capacities\n");

  std::vector<int> ptr, col;
  stencil27(40, ptr, col);  // 64,000 rows: one range
  check_tiles("27pt_40", 40 * 40 * 40, ptr, col, 3049, 1024);
  const unsigned golden = 0x9E3779B1u;
  stencil27(64, ptr, col);  // 262,144 rows: eight ranges
  check_tiles("27pt_64", 64 * 64 * 64, ptr, col, 3049, 1024);
  check_tiles("27pt_64_small_tiles", 64 * 64 * 64, ptr, col, 200, 16);
  const unsigned mul64 = choose_hash_mul(64 * 64 * 64, ptr.data(), col.data());
  if (mul64 != golden) fail("hash multiplier at 64^3 is not the golden ratio", mul64);
  std::printf("ok hash multiplier 64^3 keeps the golden ratio\n");

  // a chain of 100,003 rows: three ranges of unequal size
  {
    const int m = 100003;
    ptr.assign(m + 1, 0);
    col.clear();
    for (int r = 0; r < m; ++r) {
      for (int c = r - 1; c <= r + 1; ++c)
        if (c >= 0 && c < m) col.push_back(c);
      ptr[r + 1] = (int)col.size();
    }
    check_tiles("chain_100003", m, ptr, col, 300, 1024);
  }
  // random symmetric pattern with a few rows longer than a tile
  {
    const int m = 70001;
    std::mt19937 g(5);
    std::vector<std::vector<int>> rows(m);
    for (int r = 0; r < m; ++r) {
      rows[r].push_back(r);
      const int k = (r % 9973 == 0) ? 700 : 1 + (int)(g() % 6);
      for (int q = 0; q < k; ++q) {
        const int c = (int)(g() % m);
        rows[r].push_back(c);
        rows[c].push_back(r);
      }
    }
    ptr.assign(m + 1, 0);
    col.clear();
    for (int r = 0; r < m; ++r) {
      std::sort(rows[r].begin(), rows[r].end());
      rows[r].erase(std::unique(rows[r].begin(), rows[r].end()), rows[r].end());
      col.insert(col.end(), rows[r].begin(), rows[r].end());
      ptr[r + 1] = (int)col.size();
    }
    check_tiles("random_long_rows", m, ptr, col, 500, 1024);
  }

  // the hash multiplier: the golden ratio crowds the keys of a 108^3 coarse grid; rows longer
  // than the short-row limit are not scored
  stencil27(108, ptr, col);
  const unsigned mul108 = choose_hash_mul(108 * 108 * 108, ptr.data(), col.data());
  if (mul108 == golden || (mul108 & 1u) == 0) fail("hash multiplier at 108^3", mul108);
  std::printf("ok hash multiplier 108^3 replaces the golden ratio (0x%08x)\n", mul108);
  {
    const int m = 1000;
    std::vector<int> p2(m + 1), c2;
    for (int r = 0; r < m; ++r) {
      for (int c = 0; c < 40; ++c) c2.push_back((r + c) % m < (r + c) ? c : (r + c) % m);
      std::sort(c2.end() - 40, c2.end());
      p2[r + 1] = (int)c2.size();
    }
    if (choose_hash_mul(m, p2.data(), c2.data()) != golden) fail("hash multiplier with only long rows");
    if (choose_hash_mul(0, std::vector<int>(1, 0).data(), nullptr) != golden)
      fail("hash multiplier with no rows");
  }
  std::printf("ok hash multiplier edge cases\n");
  return 0;
}
