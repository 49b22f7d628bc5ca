// Host implementation of the C ABI in include/ptap.h: plan lifecycle, the symbolic phase
// (pattern transpose, row sizes of AP, pattern of C, row classes and owner tiles), and the
// numeric, adjoint and batched launches.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/ptap.h"
#include "host_logic.hpp"
#include "internal.hpp"

using namespace ptapk;
using namespace ptapk::host;

namespace {

thread_local int32_t g_last_hip_error = 0;

struct Failure {
  ptap_status status;
};

inline void hipck(hipError_t e) {
  if (e != hipSuccess) {
    g_last_hip_error = (int32_t)e;
    (void)hipGetLastError();
    throw Failure{PTAP_ERR_HIP};
  }
}

inline void fail(ptap_status s) { throw Failure{s}; }

// The status for the exception being handled, called inside a catch (...) block: a Failure's own,
// PTAP_ERR_OOM when host memory ran out, and PTAP_ERR_UNSUPPORTED for anything else from the
// standard library (a thread that could not start, a size beyond a container's limit), so that no
// exception crosses the C interface.
ptap_status caught_status() {
  try {
    throw;
  } catch (const Failure& f) {
    return f.status;
  } catch (const std::bad_alloc&) {
    return PTAP_ERR_OOM;
  } catch (...) {
    return PTAP_ERR_UNSUPPORTED;
  }
}

void* default_alloc(size_t bytes, void*) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}
void default_release(void* p, size_t, void*) { (void)hipFree(p); }

// Device allocations of a plan, counted for the statistics.
struct Tracker {
  ptap_allocator a{default_alloc, default_release, nullptr};
  std::map<void*, size_t> live;
  int64_t current = 0, peak = 0;

  template <class T>
  T* get(size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    bytes = (bytes + 255) / 256 * 256;
    void* p = a.alloc(bytes, a.ctx);
    if (!p) fail(PTAP_ERR_OOM);
    live[p] = bytes;
    current += (int64_t)bytes;
    peak = std::max(peak, current);
    return static_cast<T*>(p);
  }
  void put(void* p) {
    if (!p) return;
    auto it = live.find(p);
    if (it == live.end()) return;
    current -= (int64_t)it->second;
    a.release(p, it->second, a.ctx);
    live.erase(it);
  }
  void release_all() {
    for (auto& kv : live) a.release(kv.first, kv.second, a.ctx);
    live.clear();
    current = 0;
  }
};

template <class T>
std::vector<T> to_host(const T* d, size_t count, hipStream_t s) {
  std::vector<T> h(count);
  if (count) {
    hipck(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    hipck(hipStreamSynchronize(s));
  }
  return h;
}

template <class T>
void to_device(T* d, const std::vector<T>& h, hipStream_t s) {
  if (!h.empty()) {
    hipck(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    hipck(hipStreamSynchronize(s));  // h may go out of scope right after
  }
}

size_t spill_ints(const std::vector<RowClass>& cls, int per_slot_ints) {
  size_t need = 0;
  for (auto& c : cls)
    if (c.global) need = std::max(need, (size_t)kSpillWaves * c.cap * per_slot_ints);
  return need;
}

// Page-locked host memory for the symbolic phase's copies of patterns and counters.  Pinning
// costs more than the copies themselves, so buffers go back to a process-wide pool after use
// and are kept until the process ends, except those above kPinnedKeepBytes, which are freed.
// A buffer waits for its stream before it is reused, so copies still in flight on an error
// path never meet the next user.
constexpr size_t kPinnedKeepBytes = (size_t)256 << 20;
std::mutex g_pinned_mu;
std::vector<std::pair<void*, size_t>> g_pinned_free;

struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  PinnedBuf(size_t want, hipStream_t stream) : s(stream) {
    want = std::max<size_t>(want, 4096);
    {
      std::lock_guard<std::mutex> lk(g_pinned_mu);
      size_t best = g_pinned_free.size();
      for (size_t k = 0; k < g_pinned_free.size(); ++k)
        if (g_pinned_free[k].second >= want && (best == g_pinned_free.size() || g_pinned_free[k].second < g_pinned_free[best].second))
          best = k;
      if (best < g_pinned_free.size()) {
        p = g_pinned_free[best].first;
        bytes = g_pinned_free[best].second;
        g_pinned_free.erase(g_pinned_free.begin() + (long)best);
        return;
      }
    }
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      fail(PTAP_ERR_OOM);
    }
    bytes = want;
  }
  ~PinnedBuf() {
    if (!p) return;
    (void)hipStreamSynchronize(s);
    if (bytes > kPinnedKeepBytes) {
      (void)hipHostFree(p);
      return;
    }
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned_free.emplace_back(p, bytes);
  }
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

constexpr size_t kRowStoreMaxBytes = (size_t)512 << 20;  // largest row store of C's count pass

// Device-to-host copy into page-locked memory, then wait.
template <class T>
void read_back(T* host, const T* dev, size_t count, hipStream_t s) {
  if (count) hipck(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, s));
  hipck(hipStreamSynchronize(s));
}

// Host-to-device copies staged through one page-locked arena (no wait: the arena outlives the
// copies, which finish before the symbolic phase returns).  Copies that do not fit the arena
// go through to_device.
struct Uploads {
  PinnedBuf buf;
  size_t used = 0;
  Uploads(size_t bytes, hipStream_t s) : buf(bytes, s) {}
  template <class T>
  void put(T* dev, const std::vector<T>& v) {
    const size_t b = v.size() * sizeof(T);
    if (!b) return;
    if (used + b > buf.bytes) {
      to_device(dev, v, buf.s);
      return;
    }
    unsigned char* h = buf.as<unsigned char>() + used;
    memcpy(h, v.data(), b);
    hipck(hipMemcpyAsync(dev, h, b, hipMemcpyHostToDevice, buf.s));
    used = (used + b + 255) & ~(size_t)255;
  }
};

// Device classes from per-item codes (launch_class_build): the group sizes, read back after one
// wait, and the rows of all groups in one allocation (*sorted; null if no row is kept).  The
// classes built from it point into that allocation, so they are released together.
std::vector<int> classes_from_codes(Tracker& t, const int* code, const int* list, int count, int nbins,
                                    int** sorted, hipStream_t s) {
  *sorted = nullptr;
  std::vector<int> hist(nbins, 0);
  if (count <= 0) return hist;
  int* srt = t.get<int>(count);
  const size_t cells1 = class_scratch_ints(count, nbins);
  int* scr = t.get<int>(cells1);
  long long* ss = t.get<long long>(scan_scratch_count((long long)cells1 - 1));
  int* dh = t.get<int>(nbins + 1);
  hipck(launch_fill_i32(dh, 0, nbins + 1, s));
  hipck(launch_class_build(code, list, count, nbins, scr, ss, dh + nbins, srt, dh, s));
  PinnedBuf hb((nbins + 1) * sizeof(int), s);
  read_back(hb.as<int>(), dh, (size_t)nbins + 1, s);
  for (int b = 0; b < nbins; ++b) hist[b] = hb.as<int>()[b];
  const bool overflow = hb.as<int>()[nbins] != 0;
  t.put(scr);
  t.put(ss);
  t.put(dh);
  if (overflow) fail(PTAP_ERR_TOO_LARGE);
  long long kept = 0;
  for (int b = 0; b < nbins; ++b) kept += hist[b];
  if (kept == 0)
    t.put(srt);
  else
    *sorted = srt;
  return hist;
}

// Capacity classes from the groups 0..30 of a class build (group b: tables of 2^b slots).
std::vector<RowClass> cap_classes(const std::vector<int>& hist, int* sorted, int lds_max) {
  std::vector<RowClass> out;
  long long off = 0;
  for (int b = 0; b < (int)hist.size(); ++b) {
    if (hist[b] && b < 31) {
      RowClass rc;
      rc.cap = 1 << b;
      rc.global = rc.cap > lds_max;
      rc.count = hist[b];
      rc.rows = sorted + off;
      out.push_back(rc);
    }
    off += hist[b];
  }
  return out;
}

// Start of group b of a class build.
int* group_rows(const std::vector<int>& hist, int* sorted, int b) {
  long long off = 0;
  for (int q = 0; q < b; ++q) off += hist[q];
  return hist[b] ? sorted + off : nullptr;
}

// Classes by hash capacity of the rows list[0..count) (list null: rows 0..count-1), with the
// key bound need[row] (device).
template <class T>
std::vector<RowClass> make_classes_dev(Tracker& t, const T* need, const int* list, int count, int lds_max,
                                       hipStream_t s) {
  if (count <= 0) return {};
  int* code = t.get<int>(count);
  if constexpr (sizeof(T) == 8)
    hipck(launch_cap_codes_i64(need, list, count, code, s));
  else
    hipck(launch_cap_codes_i32(need, list, count, code, s));
  int* sorted = nullptr;
  const std::vector<int> hist = classes_from_codes(t, code, list, count, 31, &sorted, s);
  t.put(code);
  return cap_classes(hist, sorted, lds_max);
}

// Release the rows of a set of classes built together (one allocation, or one per class).
void put_classes(Tracker& t, std::vector<RowClass>& cls) {
  for (auto& c : cls) t.put(c.rows);
  cls.clear();
}

}  // namespace

struct ptap_plan {
  Tracker mem;
  ptap_options opt{};
  Patterns pat{};
  long long nnzA = 0, nnzP = 0;
  bool sym_done = false;
  int lds_budget = 65536;
  int lds_device = 65536;  // LDS bytes one workgroup may use on this device
  int n_cu = 256;          // compute units of this device
  int owner_waves = kFastWaves;
  int lds_hash_max = kLdsHashMax;
  int lds_keys_max = kLdsKeysMax;

  int* C_rowptr = nullptr;
  int* C_col = nullptr;
  long long nnzC = 0;

  // pattern transpose (kept by two-step only)
  int* pt_ptr = nullptr;
  int* pt_row = nullptr;
  int* pt_pos = nullptr;

  // owner fold: tiles (row lists), the slot of every row of C, per-tile fine-row lists
  int ntiles = 0, TE = 0;
  int* tile_ptr = nullptr;
  int* tile_rows = nullptr;
  int* tile_slot = nullptr;
  int* tile_fptr = nullptr;
  int* tile_fine = nullptr;
  int* off_fptr = nullptr;  // two-pass all-at-once: per tile, rows with owned off-block entries
  int* off_fine = nullptr;
  std::vector<int> host_fptr;
  std::vector<TileClass> tclasses;
  bool any_tile_global = false;
  // staged-tile kernel: the tiles that take it, their halo rows and the launch's LDS layout
  int* staged_tiles = nullptr;
  int n_staged = 0;
  int* halo_ptr = nullptr;
  int* halo_rows = nullptr;
  StagedLayout staged_L{};
  bool wide_a = false;  // A's values pass 2 GiB: the short-row owner kernel reads them by address
  unsigned hash_mul = 0x9E3779B1u;  // the short-row owner kernel's R_I hash multiplier

  // atomic fold: general row classes and the short-row lists ([0] at most 32 entries in A(I,:),
  // [1] more)
  std::vector<RowClass> arows;
  int* af_short[2] = {nullptr, nullptr};
  int n_af_short[2] = {0, 0};

  // two-step
  int* AP_rowptr = nullptr;
  int* AP_col = nullptr;
  double* AP_val = nullptr;
  double* PT_val = nullptr;
  long long nnzAP = 0;
  std::vector<RowClass> ap_rows, ptc_rows;
  // rows of AP and of C for the short-row kernel (rowmul.hip): [0] at most 32 entries in the
  // row of A (of P^T), [1] more
  int* ap_short[2] = {nullptr, nullptr};
  int* ptc_short[2] = {nullptr, nullptr};
  int n_ap_short[2] = {0, 0}, n_ptc_short[2] = {0, 0};

  // adjoint
  std::vector<RowClass> bwd_rows;

  // spill tables for numeric / adjoint launches (spill_slots keys and as many values)
  int* gtab = nullptr;
  double* gval = nullptr;
  size_t spill_slots = 0;

  // numeric cache (options.cache): packed extent of the row of P selected by each entry of A
  int* A_pext = nullptr;
  int64_t cache_bytes = 0;

  // block-sparse plans (ptap_plan_create_bsr): block size, rows of C accumulated in LDS or in C
  int bs = 1;
  int* bsr_rows_lds = nullptr;
  int* bsr_rows_glob = nullptr;
  int bsr_n_lds = 0, bsr_n_glob = 0, bsr_cap = 64, bsr_ncmax = 0;

  int fold_used = PTAP_FOLD_OWNER;
  int64_t rows_formed = 0, rows_needed = 0, fold_terms = 0, products = 0;
  double est_owner_ms = 0.0, est_atomic_ms = 0.0;  // AUTO: the fold cost model's estimates
  int64_t pattern_bytes = 0;
};

struct ptap_batch {
  Tracker mem;
  std::vector<ptap_plan*> plans;
  std::vector<int> level;
  std::vector<int> levels;                 // distinct levels, ascending
  std::vector<std::vector<int>> level_plans;
  std::vector<int2*> items;                // per level, device (plan, tile) work lists
  std::vector<int> nitems;
  int* counters = nullptr;                 // per level, one work counter per XCD
  OwnerBatchPlan* d_plans = nullptr;
  int grid = 0;
  size_t lds = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const double*> A_vals, P_vals;
  std::vector<double*> C_vals;
};

static void validate_patterns(ptap_plan* P, hipStream_t s);

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

void ptap_options_default(ptap_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->algo = PTAP_MERGED;
  o->fold = PTAP_FOLD_AUTO;
  o->nblocks = 1;
  o->tile_entries = 0;
  o->hash_slots = 0;
  o->validate = 1;
  o->xcd_remap = 1;
}

const char* ptap_status_string(ptap_status s) {
  switch (s) {
    case PTAP_OK: return "ok";
    case PTAP_ERR_INPUT: return "invalid input";
    case PTAP_ERR_TOO_LARGE: return "count overflows int32 indexing";
    case PTAP_ERR_OOM: return "out of memory (device allocator or host)";
    case PTAP_ERR_HIP: return "HIP runtime error";
    case PTAP_ERR_STATE: return "call out of order";
    case PTAP_ERR_UNSUPPORTED: return "unsupported option combination";
  }
  return "unknown status";
}

int32_t ptap_last_hip_error(void) { return g_last_hip_error; }

ptap_status ptap_stream_sum(const double* x, int64_t n, double* out, hipStream_t s) {
  if (n < 0 || !out || (n > 0 && !x) || ((uintptr_t)x & 15u)) return PTAP_ERR_INPUT;
  try {
    hipck(launch_stream_sum(x, n, out, s));
  } catch (...) {
    const ptap_status st = caught_status();
    return st;
  }
  return PTAP_OK;
}

ptap_status ptap_plan_create(ptap_plan** out, int32_t n, int32_t m, const int32_t* A_rowptr,
                             const int32_t* A_col, int64_t A_nnz, const int32_t* P_rowptr,
                             const int32_t* P_col, int64_t P_nnz, const ptap_options* opts,
                             const ptap_allocator* alloc, hipStream_t stream) {
  if (!out) return PTAP_ERR_INPUT;
  *out = nullptr;
  if (n < 0 || m < 0 || A_nnz < 0 || P_nnz < 0 || !A_rowptr || !P_rowptr) return PTAP_ERR_INPUT;
  if ((A_nnz > 0 && !A_col) || (P_nnz > 0 && !P_col)) return PTAP_ERR_INPUT;
  if (A_nnz > INT32_MAX || P_nnz > INT32_MAX) return PTAP_ERR_TOO_LARGE;
  ptap_options o;
  ptap_options_default(&o);
  if (opts) o = *opts;
  if (o.algo < PTAP_ALLATONCE || o.algo > PTAP_TWOSTEP) return PTAP_ERR_INPUT;
  if (o.fold < PTAP_FOLD_AUTO || o.fold > PTAP_FOLD_OWNER) return PTAP_ERR_INPUT;
  if (o.nblocks < 1 || o.tile_entries < 0 || o.hash_slots < 0 || o.tile_lds < 0) return PTAP_ERR_INPUT;
  if (o.owner_kernel < 0 || o.owner_kernel > 1) return PTAP_ERR_INPUT;
  if (o.validate < 0 || o.validate > 2) return PTAP_ERR_INPUT;
  if (o.hash_mul != 0 && (o.hash_mul & 1u) == 0) return PTAP_ERR_INPUT;
  if (o.owner_waves != 0 && o.owner_waves != 4 && o.owner_waves != 8 && o.owner_waves != 16)
    return PTAP_ERR_INPUT;
  if (o.hash_slots && (o.hash_slots < 64 || (o.hash_slots & (o.hash_slots - 1)))) return PTAP_ERR_INPUT;
  if (alloc && (!alloc->alloc || !alloc->release)) return PTAP_ERR_INPUT;

  ptap_plan* p = new (std::nothrow) ptap_plan();
  if (!p) return PTAP_ERR_OOM;
  if (alloc) p->mem.a = *alloc;
  p->opt = o;
  p->pat = Patterns{n, m, A_rowptr, A_col, P_rowptr, P_col};
  p->nnzA = A_nnz;
  p->nnzP = P_nnz;
  try {
    int dev = 0, lds = 0;
    hipck(hipGetDevice(&dev));
    hipck(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    p->lds_budget = std::min(lds, 65536);
    p->lds_device = lds;
    int cus = 0;
    hipck(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    p->n_cu = std::max(1, cus);
    if (o.hash_slots) {
      p->lds_hash_max = std::min(p->lds_hash_max, (int)o.hash_slots);
      p->lds_keys_max = std::min(p->lds_keys_max, (int)o.hash_slots);
    }
    if (o.validate) validate_patterns(p, stream);
  } catch (...) {
    const ptap_status st = caught_status();
    p->mem.release_all();
    delete p;
    return st;
  }
  *out = p;
  return PTAP_OK;
}

ptap_status ptap_plan_create_bsr(ptap_plan** out, int32_t nb, int32_t mb, int32_t bs,
                                 const int32_t* A_rowptr, const int32_t* A_col, int64_t A_nnzb,
                                 const int32_t* P_rowptr, const int32_t* P_col, int64_t P_nnzb,
                                 const ptap_options* opts, const ptap_allocator* alloc,
                                 hipStream_t stream) {
  if (!out) return PTAP_ERR_INPUT;
  *out = nullptr;
  if (bs < 1 || bs > kBsrMaxBlock) return PTAP_ERR_INPUT;
  ptap_options o;
  ptap_options_default(&o);
  if (opts) o = *opts;
  if (o.algo == PTAP_TWOSTEP || o.backward) return PTAP_ERR_UNSUPPORTED;
  if ((A_nnzb + 1) * bs * bs > (int64_t)1 << 40 || (P_nnzb + 1) * bs * bs > (int64_t)1 << 40)
    return PTAP_ERR_TOO_LARGE;
  o.fold = PTAP_FOLD_OWNER;
  o.cache = 0;
  ptap_status st = ptap_plan_create(out, nb, mb, A_rowptr, A_col, A_nnzb, P_rowptr, P_col, P_nnzb, &o,
                                    alloc, stream);
  if (st == PTAP_OK) (*out)->bs = bs;
  return st;
}

static void validate_patterns(ptap_plan* P, hipStream_t s) {
  const Patterns& pat = P->pat;
  // [0] error bits, [1..4] two pairs of descent counts (A, P)
  int* err = P->mem.get<int>(10);
  hipck(launch_fill_i32(err, 0, 10, s));
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(err + 2);
  hipck(launch_validate_pattern(pat.A_rowptr, pat.A_col, pat.n, pat.n, P->nnzA, err, cnt, s));
  hipck(launch_validate_pattern(pat.P_rowptr, pat.P_col, pat.n, pat.m, P->nnzP, err, cnt + 2, s));
  PinnedBuf hb(10 * sizeof(int), s);
  read_back(hb.as<int>(), err, 10, s);
  P->mem.put(err);
  const unsigned long long* hc = reinterpret_cast<const unsigned long long*>(hb.as<int>() + 2);
  if (hb.as<int>()[0] || hc[0] != hc[1] || hc[2] != hc[3]) fail(PTAP_ERR_INPUT);
}

static void symbolic_impl(ptap_plan* P, hipStream_t s) {
  Tracker& t = P->mem;
  const Patterns& pat = P->pat;
  const int n = pat.n, m = pat.m;
  const bool two = P->opt.algo == PTAP_TWOSTEP;
  const bool blk = P->bs > 1;
  // The patterns are caller-owned; with validation 1 they are checked again right before use,
  // so that arrays changed or released since plan creation are reported instead of read (2: the
  // caller runs this right after creating the plan, whose check still holds).
  if (P->opt.validate == 1) validate_patterns(P, s);
  // device counters read back together: [0] a scan total passed INT32_MAX, [1] rows of AP left
  // to the class launches, [2] rows of C left to them; [4..5] a scan's 64-bit total (copied)
  int* dflag = t.get<int>(8);
  hipck(launch_fill_i32(dflag, 0, 8, s));
  PinnedBuf small(4096, s);
  int* hsm = small.as<int>();
  auto scan = [&](const int* in, long long count, int* out) {
    long long* sc = t.get<long long>(scan_scratch_count(count));
    hipck(launch_scan_i32(in, count, out, sc, dflag, s));
    hipck(hipMemcpyAsync(dflag + 4, sc + (scan_scratch_count(count) - 1), sizeof(long long),
                         hipMemcpyDeviceToDevice, s));
    t.put(sc);
  };

  // --- Column index lists of P (pattern transpose; integer only, no values).
  P->pt_ptr = t.get<int>(m + 1);
  P->pt_row = t.get<int>(P->nnzP);
  P->pt_pos = (two || blk) ? t.get<int>(P->nnzP) : nullptr;
  {
    int* cnt = t.get<int>(m + 1);
    hipck(launch_fill_i32(cnt, 0, m + 1, s));
    hipck(launch_count_cols(pat.P_col, P->nnzP, cnt, s));
    scan(cnt, m, P->pt_ptr);
    if (m) hipck(hipMemcpyAsync(cnt, P->pt_ptr, (size_t)m * sizeof(int), hipMemcpyDeviceToDevice, s));
    hipck(launch_transpose_fill(pat.P_rowptr, pat.P_col, n, cnt, P->pt_row, P->pt_pos, s));
    t.put(cnt);
  }

  // --- |R_I| and w_I for every fine row (Alg. 1 / 2) in one pass; rows whose products could
  // outgrow its table go to launches by capacity class, sized by w_I.
  // |R_I|, w_I and the rows the one-pass table cannot hold; allocated when R_I is formed (after
  // C's row store is released where R_I comes late), so the two are never held together
  int* r = nullptr;
  int* w = nullptr;
  int* ap_ovf = nullptr;
  int* c_cnt = nullptr;
  unsigned char* c_flag = nullptr;
  int* c_ovf = nullptr;
  int* c_store = nullptr;  // rows of C of at most kRowStore columns, sorted, from the count pass
  int n_c_ovf = 0;
  int rmax_all = 0, pmax_all = 0;
  // merged / all-at-once with tiles to grow: C's fill pass runs range by range in the owner branch,
  // and |R_I| is formed on the device while the host grows the tiles
  const bool fill_by_range = !two && !blk && P->opt.fold != PTAP_FOLD_ATOMIC;
  bool r_done = false;
  // Counters for the statistics (rows needed, fold terms sum_I nnz(P(I,:)) |R_I|, longest rows,
  // products), reduced on the device once |R_I| is known; read back into hsm[8..17].
  unsigned long long* st = t.get<unsigned long long>(5);
  hipck(launch_fill_i32(reinterpret_cast<int*>(st), 0, 10, s));
  auto launch_r = [&] {
    r = t.get<int>(n);
    w = t.get<int>(n);
    ap_ovf = t.get<int>(n);
    hipck(launch_ap_count(pat, r, w, ap_ovf, dflag + 1, s));
  };
  // after a read of dflag: rows the one-pass table could not hold, then the statistics
  auto finish_r = [&](int novf) {
    if (novf > 0) {
      std::vector<RowClass> cls = make_classes_dev(t, w, ap_ovf, novf, P->lds_keys_max, s);
      size_t gi = spill_ints(cls, 2);  // keys + list (cap/2), rounded up
      int* gtab = gi ? t.get<int>(gi) : nullptr;
      for (auto& c : cls) hipck(launch_ap_row_count(pat, c, r, gtab, s));
      put_classes(t, cls);
      t.put(gtab);
    }
    t.put(ap_ovf);
    hipck(launch_row_stats(pat, r, w, st, s));
    t.put(w);
    hipck(hipMemcpyAsync(hsm + 8, st, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    r_done = true;
  };
  // after the read that follows finish_r
  auto take_stats = [&](bool bounds_too) {
    unsigned long long h[5];
    memcpy(h, hsm + 8, sizeof(h));
    P->rows_needed = (long long)h[0];
    P->fold_terms = (long long)h[1];
    P->products = (long long)h[4];
    if (bounds_too) {
      rmax_all = (int)h[2];
      pmax_all = (int)h[3];
    }
  };
  if (!fill_by_range) launch_r();
  // --- Merged / all-at-once: count pass of C's pattern by the two-level union (needs no R_I)
  if (!two) {
    c_cnt = t.get<int>(m + 1);
    c_flag = t.get<unsigned char>(m);
    c_ovf = t.get<int>(m);
    // (the store is skipped where it would pass kRowStoreMaxBytes: those rows take the fill pass)
    if ((size_t)m * kRowStore * sizeof(int) <= kRowStoreMaxBytes) c_store = t.get<int>((size_t)m * kRowStore);
    hipck(launch_c_two_level(pat, P->pt_ptr, P->pt_row, false, c_cnt, c_flag, c_ovf, dflag + 2,
                             nullptr, nullptr, c_store, dflag + 3, 0, m, s));
  }
  read_back(hsm, dflag, 4, s);
  if (hsm[0]) fail(PTAP_ERR_TOO_LARGE);
  n_c_ovf = hsm[2];
  const int n_c_fill = hsm[3];  // rows of C longer than the row store holds
  // C's columns for rows [lo, hi) once the row pointers are known: the fill pass for rows longer
  // than the row store, a copy for the others
  auto fill_c = [&](int lo, int hi) {
    if (n_c_fill > 0)
      hipck(launch_c_two_level(pat, P->pt_ptr, P->pt_row, true, nullptr, c_flag, nullptr, nullptr, P->C_rowptr,
                               P->C_col, nullptr, nullptr, lo, hi, s));
    if (c_store) hipck(launch_c_from_store(P->C_rowptr, c_store, c_flag, lo, hi, P->C_col, s));
  };
  if (fill_by_range && n_c_ovf > 0) {
    // the rows of C the union left are sized by sum |R_I|: form R_I now
    launch_r();
    read_back(hsm, dflag, 4, s);
  }
  if (!fill_by_range || n_c_ovf > 0) finish_r(hsm[1]);

  // --- Two-step: the stored pattern of AP (rows sorted).
  if (two) {
    P->AP_rowptr = t.get<int>(n + 1);
    scan(r, n, P->AP_rowptr);
    read_back(hsm, dflag, 6, s);
    if (hsm[0]) fail(PTAP_ERR_TOO_LARGE);
    long long acc;
    memcpy(&acc, hsm + 4, sizeof(acc));
    P->nnzAP = acc;
    P->AP_col = t.get<int>(acc);
    P->ap_rows = make_classes_dev(t, r, nullptr, n, P->lds_keys_max, s);
    size_t gi = spill_ints(P->ap_rows, 2);
    int* gtab = gi ? t.get<int>(gi) : nullptr;
    for (auto& c : P->ap_rows) hipck(launch_ap_row_fill(pat, c, P->AP_rowptr, P->AP_col, gtab, s));
    t.put(gtab);
    put_classes(t, P->ap_rows);
  }

  // --- Pattern of C by rows: counts, scan (the one read of nnz(C)), fill.
  {
    if (two) {
      // the union of the stored rows of AP under column i of P, tables sized by sum |R_I|
      c_cnt = t.get<int>(m + 1);
      long long* bound = t.get<long long>(m);
      hipck(launch_c_bound(P->pt_ptr, P->pt_row, r, m, bound, s));
      std::vector<RowClass> cls = make_classes_dev(t, bound, nullptr, m, P->lds_keys_max, s);
      t.put(bound);
      size_t gi = spill_ints(cls, 2);
      int* gtab = gi ? t.get<int>(gi) : nullptr;
      hipck(launch_fill_i32(c_cnt, 0, m, s));
      for (auto& c : cls)
        hipck(launch_c_rows(pat, P->pt_ptr, P->pt_row, P->AP_rowptr, P->AP_col, c, false, c_cnt, nullptr,
                            nullptr, gtab, s));
      put_classes(t, cls);
      t.put(gtab);
    } else if (n_c_ovf > 0) {
      // rows the two-level union left: tables sized by sum |R_I|
      long long* bound = t.get<long long>(m);
      hipck(launch_c_bound_list(P->pt_ptr, P->pt_row, r, c_ovf, n_c_ovf, m, bound, s));
      std::vector<RowClass> cls = make_classes_dev(t, bound, c_ovf, n_c_ovf, P->lds_keys_max, s);
      t.put(bound);
      size_t gi = spill_ints(cls, 2);
      int* gtab = gi ? t.get<int>(gi) : nullptr;
      for (auto& c : cls)
        hipck(launch_c_rows(pat, P->pt_ptr, P->pt_row, nullptr, nullptr, c, false, c_cnt, nullptr, nullptr,
                            gtab, s));
      put_classes(t, cls);
      t.put(gtab);
    }
    P->C_rowptr = t.get<int>(m + 1);
    scan(c_cnt, m, P->C_rowptr);
    unsigned* bnd = nullptr;
    if (!r_done) {
      // the tile size needs bounds on |R_I| and the row lengths before R_I is formed
      bnd = t.get<unsigned>(2);
      hipck(launch_fill_i32(reinterpret_cast<int*>(bnd), 0, 2, s));
      hipck(launch_row_bounds(pat, P->C_rowptr, bnd, s));
      hipck(hipMemcpyAsync(hsm + 20, bnd, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    }
    read_back(hsm, dflag, 6, s);
    if (hsm[0]) fail(PTAP_ERR_TOO_LARGE);
    if (r_done) {
      take_stats(true);
    } else {
      rmax_all = hsm[20];
      pmax_all = hsm[21];
      t.put(bnd);
    }
    long long acc;
    memcpy(&acc, hsm + 4, sizeof(acc));
    P->nnzC = acc;
    P->C_col = t.get<int>(acc);
    if (two) {
      std::vector<RowClass> cls = make_classes_dev(t, c_cnt, nullptr, m, P->lds_keys_max, s);
      size_t gi = spill_ints(cls, 2);
      int* gtab = gi ? t.get<int>(gi) : nullptr;
      for (auto& c : cls)
        hipck(launch_c_rows(pat, P->pt_ptr, P->pt_row, P->AP_rowptr, P->AP_col, c, true, nullptr, P->C_rowptr,
                            P->C_col, gtab, s));
      put_classes(t, cls);
      t.put(gtab);
    } else {
      // rows the two-level union left first; the others here, or by row range in the owner branch
      // below, where each range's tiles grow on the host as soon as its rows are filled and copied
      if (n_c_ovf > 0) {
        std::vector<RowClass> cls = make_classes_dev(t, c_cnt, c_ovf, n_c_ovf, P->lds_keys_max, s);
        size_t gi = spill_ints(cls, 2);
        int* gtab = gi ? t.get<int>(gi) : nullptr;
        for (auto& c : cls)
          hipck(launch_c_rows(pat, P->pt_ptr, P->pt_row, nullptr, nullptr, c, true, nullptr, P->C_rowptr,
                              P->C_col, gtab, s));
        put_classes(t, cls);
        t.put(gtab);
      }
      if (!fill_by_range) fill_c(0, m);
    }
    t.put(c_cnt);
    t.put(c_ovf);
    if (!fill_by_range) {
      t.put(c_store);
      c_store = nullptr;
    }
    P->pattern_bytes = (int64_t)(m + 1 + acc) * (int64_t)sizeof(int);
  }

  size_t spill_need_ints = 0, spill_need_vals = 0;
  const int lmax = P->lds_hash_max;

  if (blk) {
    // Block rows: the row form, one workgroup per row of C (bsr.hip).  Rows whose accumulators
    // fit the LDS target are summed in LDS; longer rows add into C with device atomics.
    P->fold_used = PTAP_FOLD_OWNER;
    P->rows_formed = P->nnzP;  // a fine block row is formed once per block of its row of P
    PinnedBuf cb(((size_t)m + 1) * sizeof(int), s);
    read_back(cb.as<int>(), P->C_rowptr, (size_t)m + 1, s);
    const int* h_c_ptr = cb.as<int>();
    const size_t target = std::min<size_t>((size_t)P->lds_device, 65536);
    int ncmax = 0;
    std::vector<int> lrows, grows;
    for (int i = 0; i < m; ++i) {
      const int nc = h_c_ptr[i + 1] - h_c_ptr[i];
      if (nc == 0) continue;
      if (bsr_lds_bytes(P->bs, cap_for(nc), nc, true) <= target) {
        lrows.push_back(i);
        ncmax = std::max(ncmax, nc);
      } else {
        grows.push_back(i);
      }
    }
    P->bsr_ncmax = ncmax;
    P->bsr_cap = cap_for(std::max(ncmax, 1));
    if (bsr_lds_bytes(P->bs, P->bsr_cap, ncmax, true) > (size_t)P->lds_device) fail(PTAP_ERR_UNSUPPORTED);
    P->bsr_n_lds = (int)lrows.size();
    P->bsr_n_glob = (int)grows.size();
    if (!lrows.empty()) {
      P->bsr_rows_lds = t.get<int>(lrows.size());
      to_device(P->bsr_rows_lds, lrows, s);
    }
    if (!grows.empty()) {
      P->bsr_rows_glob = t.get<int>(grows.size());
      to_device(P->bsr_rows_glob, grows, s);
    }
  } else if (two) {
    P->fold_used = PTAP_FOLD_AUTO;
    P->AP_val = t.get<double>(P->nnzAP);
    P->PT_val = t.get<double>(P->nnzP);
    // Rows with at most 32 entries in AP(I,:) (in C(i,:) for the second product) take the
    // short-row kernel when every array fits its byte range; the others go by capacity class.
    RowMulArgs g1{}, g2{};
    g1.nX = g1.nY = g2.nY = n;  // A and P have n rows, P^T has m
    g2.nX = m;
    g1.nnzX = P->nnzA;
    g1.nnzY = g2.nnzX = P->nnzP;
    g1.nnzO = g2.nnzY = P->nnzAP;
    g2.nnzO = P->nnzC;
    const bool short_ok = rowmul_short_fits(g1) && rowmul_short_fits(g2);
    int* code = t.get<int>(std::max(n, m));
    hipck(launch_rowform_codes(0, n, r, pat.A_rowptr, nullptr, nullptr, nullptr, short_ok, code, s));
    int* sa = nullptr;
    const std::vector<int> ha = classes_from_codes(t, code, nullptr, n, kCodeShort1 + 1, &sa, s);
    hipck(launch_rowform_codes(1, m, nullptr, P->pt_ptr, P->C_rowptr, nullptr, nullptr, short_ok, code, s));
    int* sc = nullptr;
    const std::vector<int> hc = classes_from_codes(t, code, nullptr, m, kCodeShort1 + 1, &sc, s);
    t.put(code);
    P->ap_rows = cap_classes(ha, sa, lmax);
    P->ptc_rows = cap_classes(hc, sc, lmax);
    long long kept = 0;
    for (int v : ha) kept += v;
    for (int k = 0; k < 2; ++k) {
      P->n_ap_short[k] = ha[kCodeShort0 + k];
      P->ap_short[k] = group_rows(ha, sa, kCodeShort0 + k);
      P->n_ptc_short[k] = hc[kCodeShort0 + k];
      P->ptc_short[k] = group_rows(hc, sc, kCodeShort0 + k);
    }
    spill_need_ints = std::max(spill_ints(P->ap_rows, 1), spill_ints(P->ptc_rows, 1));
    spill_need_vals = spill_need_ints;
    P->rows_formed = kept;
  } else {
    // AUTO: build the owner fold's tiles, then keep them or take the atomic fold after all,
    // whichever the cost model of the two folds (host_logic.hpp fold_estimate) estimates faster.
    bool atomic = P->opt.fold == PTAP_FOLD_ATOMIC;
    if (!atomic) {
      // C's pattern on the host for growing the tiles (page-locked memory): the row pointers
      // first, then the columns (filled at once) copied range by range, each range's tiles
      // growing as soon as its columns have arrived
      PinnedBuf cbuf(((size_t)m + 1 + (size_t)P->nnzC) * sizeof(int), s);
      int* h_c_ptr = cbuf.as<int>();
      int* h_c_col = h_c_ptr + m + 1;
      read_back(h_c_ptr, P->C_rowptr, (size_t)m + 1, s);
      const int nparts = grow_parts(m);
      fill_c(0, m);
      t.put(c_store);
      c_store = nullptr;
      std::vector<hipEvent_t> arrived(nparts, nullptr);
      struct EventsGuard {
        std::vector<hipEvent_t>& e;
        ~EventsGuard() {
          for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } events_guard{arrived};
      for (int q = 0; q < nparts; ++q) {
        int lo, hi;
        grow_range_bounds(m, nparts, q, lo, hi);
        const size_t b = (size_t)h_c_ptr[lo], e = (size_t)h_c_ptr[hi];
        if (e > b)
          hipck(hipMemcpyAsync(h_c_col + b, P->C_col + b, (e - b) * sizeof(int), hipMemcpyDeviceToHost, s));
        hipck(hipEventCreateWithFlags(&arrived[q], hipEventDisableTiming));
        hipck(hipEventRecord(arrived[q], s));
      }
      // Tiles of rows of C held in LDS.  Tiles whose fine rows are short (|R_I| and
      // the rows of P within the short-row limits) take the short-row kernel; the tile size is
      // set by that kernel's LDS layout when every row qualifies.
      // the short-row kernel addresses P's arrays, A's columns and the row pointers with 32-bit
      // byte offsets, and A's values so too while they stay under 2 GiB (by address beyond)
      const bool fast_fits = P->nnzP * 8 < (1LL << 31) && P->nnzA * 4 < (1LL << 31) &&
                             ((long long)n + 1) * 4 < (1LL << 31);
      P->wide_a = P->nnzA * 8 >= (1LL << 31);
      const bool fast_all = fast_fits && rmax_all <= kFastMaxKeys && pmax_all <= kFastMaxKeys;
      const int nw = P->opt.owner_waves ? P->opt.owner_waves : kFastWaves;
      if (nw != 4 && nw != 8 && nw != 16) fail(PTAP_ERR_INPUT);
      P->owner_waves = nw;
      const int lds_tile = std::min(P->lds_device, P->opt.tile_lds ? P->opt.tile_lds : kTileLdsTarget);
      const int TR = kTileRows;
      const int cap_all = std::min(cap_for(rmax_all), lmax);
      long long room;
      // (256 bytes stay free for the batched kernel's own LDS variables, so that two workgroups
      // still fit in a CU's 160 KiB)
      if (fast_all)
        room = ((long long)lds_tile - (long long)nw * (long long)owner_fast_wave_bytes() - (TR + 1) * 4LL - 16 -
                256) / 12;
      else
        room = ((long long)lds_tile - (long long)kWavesPerBlock * ((long long)sizeof(WaveScratch) + (long long)cap_all * 12) -
                (TR + 1) * 4LL - 16) / 12;
      int TE = (int)std::max<long long>(16, room);
      // the staged-tile kernel (merged or one-block forms, A's values within 2 GiB) holds a tile's
      // halo rows of P beside the tile: smaller tiles, one workgroup per CU
      const bool twopass_owner = P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1;
      int crow_max = 0;
      for (int i = 0; i < m; ++i) crow_max = std::max(crow_max, h_c_ptr[i + 1] - h_c_ptr[i]);
      const bool staging = P->opt.owner_kernel == 1 && !twopass_owner && fast_fits && !P->wide_a &&
                           !P->opt.cache && crow_max <= kStagedMaxRank;
      if (staging && !P->opt.tile_lds) TE = std::min(TE, kStagedTileEntries);
      if (P->opt.tile_entries) {
        TE = std::min(TE, (int)P->opt.tile_entries);
      } else if (!P->opt.tile_lds) {
        // Fewer tiles than resident workgroups (two per CU) leave CUs idle: shrink the tiles until
        // they fill about 95% of one round of workgroups (not more, or a few tiles run alone in
        // a second round), accepting the extra rows of AP that smaller tiles form twice.
        const long long slots = (staging ? 1LL : 2LL) * P->n_cu;
        if (P->nnzC / TE < slots) {
          const long long te_par = (P->nnzC * 100) / (95 * slots);
          TE = (int)std::min<long long>(TE, std::max<long long>(te_par, 256));
        }
      }
      P->TE = TE;
      std::vector<int> tptr, trows;
      std::vector<char> tglob;
      // |R_I| on the device while the tiles grow on the host
      if (!r_done) launch_r();
      std::atomic<int> copy_err{0};
      grow_tiles(m, h_c_ptr, h_c_col, TE, TR, tptr, trows, tglob, [&](int q) {
        if (hipEventSynchronize(arrived[q]) != hipSuccess) copy_err = 1;
      });
      if (copy_err) hipck(hipErrorUnknown);
      const bool stats_pending = !r_done;
      if (!r_done) {
        read_back(hsm, dflag, 4, s);
        finish_r(hsm[1]);
      }
      // the hash multiplier is chosen on a thread of its own while the device works on the tiles
      std::exception_ptr mul_err;
      std::thread mul_thread;
      auto pick_mul = [&] {
        try {
          P->hash_mul = choose_hash_mul(m, h_c_ptr, h_c_col);
        } catch (...) {
          mul_err = std::current_exception();
        }
      };
      if (P->opt.hash_mul) {
        P->hash_mul = P->opt.hash_mul;
      } else {
        try {
          mul_thread = std::thread(pick_mul);
        } catch (...) {
          pick_mul();  // no thread to spare
        }
      }
      struct Joiner {
        std::thread& th;
        ~Joiner() {
          if (th.joinable()) th.join();
        }
      } mul_join{mul_thread};
      const int T = (int)tglob.size();
      if (T >= (1 << (31 - kTileRowBits))) fail(PTAP_ERR_TOO_LARGE);
      Uploads up(((size_t)T + 1 + (size_t)m) * sizeof(int) + 2 * (size_t)T * sizeof(int) + 65536, s);
      P->ntiles = T;
      P->tile_ptr = t.get<int>(T + 1);
      P->tile_rows = t.get<int>(m);
      P->tile_slot = t.get<int>(m);
      up.put(P->tile_ptr, tptr);
      up.put(P->tile_rows, trows);
      hipck(launch_fill_i32(P->tile_slot, -1, m, s));
      hipck(launch_tile_slot(P->tile_ptr, P->tile_rows, T, P->tile_slot, s));
      const TileSet ts{P->tile_ptr, P->tile_rows, P->tile_slot};
      // fine rows of every tile: counts (and the largest |R_I| and row lengths), a scan, the fill
      int* tcnt = t.get<int>(T + 1);
      int* trmax = t.get<int>(2 * (size_t)T);
      hipck(launch_tile_fine(pat, P->pt_ptr, P->pt_row, ts, T, r, false, tcnt, trmax, nullptr,
                             nullptr, PART_ALL, P->opt.nblocks, s));
      P->tile_fptr = t.get<int>(T + 1);
      scan(tcnt, T, P->tile_fptr);
      PinnedBuf tb((3 * (size_t)T + 1) * sizeof(int), s);
      hipck(hipMemcpyAsync(tb.as<int>(), P->tile_fptr, ((size_t)T + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
      if (T) hipck(hipMemcpyAsync(tb.as<int>() + T + 1, trmax, 2 * (size_t)T * sizeof(int), hipMemcpyDeviceToHost, s));
      read_back(hsm, dflag, 1, s);
      if (hsm[0]) fail(PTAP_ERR_TOO_LARGE);
      if (stats_pending) take_stats(false);
      t.put(tcnt);
      t.put(trmax);
      std::vector<int> fptr(tb.as<int>(), tb.as<int>() + T + 1);
      const int* hrmax = tb.as<int>() + T + 1;
      const long long acc = fptr[T];
      P->tile_fine = t.get<int>(acc);
      P->host_fptr = fptr;
      hipck(launch_tile_fine(pat, P->pt_ptr, P->pt_row, ts, T, r, true, nullptr, nullptr,
                             P->tile_fptr, P->tile_fine, PART_ALL, P->opt.nblocks, s));
      P->rows_formed = acc;
      // two-pass all-at-once (Alg. 8): the first pass walks only each tile's rows that own an
      // off-block entry there
      if (P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1) {
        int* ocnt = t.get<int>(T + 1);
        int* ormax = t.get<int>(2 * (size_t)T);
        hipck(launch_tile_fine(pat, P->pt_ptr, P->pt_row, ts, T, r, false, ocnt, ormax, nullptr,
                               nullptr, PART_OFF, P->opt.nblocks, s));
        P->off_fptr = t.get<int>(T + 1);
        scan(ocnt, T, P->off_fptr);
        read_back(hsm, dflag, 6, s);
        t.put(ocnt);
        t.put(ormax);
        long long oacc;
        memcpy(&oacc, hsm + 4, sizeof(oacc));  // at most acc, which fits
        P->off_fine = t.get<int>(oacc);
        hipck(launch_tile_fine(pat, P->pt_ptr, P->pt_row, ts, T, r, true, nullptr, nullptr,
                               P->off_fptr, P->off_fine, PART_OFF, P->opt.nblocks, s));
        P->rows_formed += oacc;
      }
      // staged tiles: halo sizes of every tile on the device, then the tiles that fit one launch
      std::vector<char> is_staged(T, 0);
      if (staging) {
        std::vector<int> all(T);
        for (int k = 0; k < T; ++k) all[k] = k;
        int* d_all = t.get<int>(T);
        to_device(d_all, all, s);
        int* st = t.get<int>(6 * (size_t)T);
        hipck(launch_tile_halo(pat, d_all, T, P->tile_fptr, P->tile_fine, false, st, nullptr,
                               nullptr, s));
        const std::vector<int> hs = to_host(st, 6 * (size_t)T, s);
        t.put(st);
        // candidate tiles and their own LDS needs
        std::vector<std::pair<size_t, int>> cand;
        std::vector<StagedCaps> caps(T);
        for (int k = 0; k < T; ++k) {
          const int* o = &hs[6 * (size_t)k];
          const int nrk = tptr[k + 1] - tptr[k];
          int rowmax = 0, te = 0;
          for (int q = tptr[k]; q < tptr[k + 1]; ++q) {
            const int len = h_c_ptr[trows[q] + 1] - h_c_ptr[trows[q]];
            rowmax = std::max(rowmax, len);
            te += len;
          }
          const bool ok = !tglob[k] && o[5] == 0 && o[0] <= kStagedMaxHalo && o[2] <= kStagedMaxCols &&
                          o[3] <= kStagedMaxA && o[4] <= kStagedMaxP && rowmax <= kStagedMaxRank &&
                          nrk <= kStagedMaxRows && o[1] < (1 << 24) && te < 65536;
          if (!ok) continue;
          caps[k] = StagedCaps{nrk, std::max(te, 1), std::max(o[0], 1), std::max(o[1], 1), std::max(o[2], 1)};
          cand.emplace_back(staged_layout(caps[k], kStagedWaves, nullptr), k);
        }
        // the launch's layout takes the maxima over its tiles: drop the largest tiles until it fits
        std::sort(cand.begin(), cand.end());
        const size_t limit = (size_t)P->lds_device - 256;  // the kernel's own LDS variables
        size_t keep = cand.size();
        StagedCaps cm{1, 1, 1, 1, 1};
        while (keep > 0) {
          cm = StagedCaps{1, 1, 1, 1, 1};
          for (size_t x = 0; x < keep; ++x) {
            const StagedCaps& c = caps[cand[x].second];
            cm.NR = std::max(cm.NR, c.NR);
            cm.TE = std::max(cm.TE, c.TE);
            cm.NH = std::max(cm.NH, c.NH);
            cm.SE = std::max(cm.SE, c.SE);
            cm.UL = std::max(cm.UL, c.UL);
          }
          if (staged_layout(cm, kStagedWaves, nullptr) <= limit) break;
          keep = keep * 31 / 32;
        }
        if (keep > 0) {
          staged_layout(cm, kStagedWaves, &P->staged_L);
          std::vector<int> stl, hptr(T + 1, 0);
          for (size_t x = 0; x < keep; ++x) is_staged[cand[x].second] = 1;
          long long hacc = 0;
          for (int k = 0; k < T; ++k) {
            if (is_staged[k]) {
              stl.push_back(k);
              hacc += hs[6 * (size_t)k];
            }
            if (hacc > INT32_MAX) fail(PTAP_ERR_TOO_LARGE);
            hptr[k + 1] = (int)hacc;
          }
          P->n_staged = (int)stl.size();
          P->staged_tiles = t.get<int>(stl.size());
          to_device(P->staged_tiles, stl, s);
          P->halo_ptr = t.get<int>(T + 1);
          to_device(P->halo_ptr, hptr, s);
          P->halo_rows = t.get<int>(std::max<long long>(hacc, 1));
          hipck(launch_tile_halo(pat, P->staged_tiles, P->n_staged, P->tile_fptr, P->tile_fine, true,
                                 nullptr, P->halo_ptr, P->halo_rows, s));
        }
        t.put(d_all);
      }
      // classes by (kernel, hash capacity, placement); a tile with no fine row still runs so that
      // its (empty) rows are written
      std::map<std::tuple<int, int, int>, std::vector<int>> groups;
      for (int k = 0; k < T; ++k) {
        if (is_staged[k]) continue;
        const int rm = hrmax[2 * k], lm = hrmax[2 * k + 1];
        const bool fast = fast_fits && !tglob[k] && rm <= kFastMaxKeys && lm <= kFastMaxKeys &&
                          owner_fast_lds_bytes(TE, nw) <= (size_t)P->lds_device;
        const int cap = cap_for(std::max(rm, 1));
        int tg = tglob[k];
        if (!fast && !tg && owner_general_lds_bytes(TE, cap, cap > lmax, false) > (size_t)P->lds_device)
          tg = 1;
        if (tg && tptr[k + 1] - tptr[k] != 1) fail(PTAP_ERR_UNSUPPORTED);  // a device-memory tile holds one row
        // short-row tiles with a row of C of more than 64 columns fold those rows key by key
        int long_c = 0;
        if (fast)
          for (int q = tptr[k]; q < tptr[k + 1] && !long_c; ++q)
            long_c = h_c_ptr[trows[q] + 1] - h_c_ptr[trows[q]] > 2 * kHalfLanes ? 1 : 0;
        groups[std::make_tuple(fast ? 1 : 0, fast ? long_c : cap, tg)].push_back(k);
      }
      for (auto& kv : groups) {
        TileClass tc;
        tc.fast = std::get<0>(kv.first) != 0;
        tc.long_c = tc.fast && std::get<1>(kv.first) != 0;
        tc.cap = tc.fast ? 64 : std::get<1>(kv.first);
        tc.hash_global = !tc.fast && tc.cap > lmax;
        tc.tile_global = std::get<2>(kv.first) != 0;
        tc.count = (int)kv.second.size();
        tc.tiles = t.get<int>(tc.count);
        up.put(tc.tiles, kv.second);
        tc.host_tiles = kv.second;
        // the short-row kernel pairs consecutive rows of a tile's list: order them by owned count
        if (tc.fast) {
          hipck(launch_tile_order(pat, tc.tiles, tc.count, P->tile_fptr, P->tile_fine, P->tile_slot, s));
          if (P->off_fptr)
            hipck(launch_tile_order(pat, tc.tiles, tc.count, P->off_fptr, P->off_fine, P->tile_slot, s));
        }
        if (tc.tile_global) P->any_tile_global = true;
        if (tc.hash_global)
          spill_need_ints = std::max(spill_need_ints, (size_t)tc.count * kWavesPerBlock * tc.cap);
        P->tclasses.push_back(tc);
      }
      if (mul_thread.joinable()) mul_thread.join();
      if (mul_err) std::rethrow_exception(mul_err);
      spill_need_vals = spill_need_ints;
      // numeric cache: only the short-row kernel reads it; the start must fit in 26 bits
      bool any_fast = false;
      for (const auto& tc : P->tclasses) any_fast = any_fast || tc.fast;
      if (P->opt.cache && any_fast && P->nnzP < (1LL << 26) && P->nnzA > 0) {
        P->A_pext = t.get<int>((size_t)P->nnzA);
        hipck(launch_pext(pat, P->nnzA, P->A_pext, s));
        P->cache_bytes = P->nnzA * (int64_t)sizeof(int);
      }
      t.put(P->pt_ptr);
      t.put(P->pt_row);
      P->pt_ptr = P->pt_row = nullptr;
      if (P->opt.fold == PTAP_FOLD_AUTO) {
        const bool twopass_fold = P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1;
        const host::FoldEstimate est = host::fold_estimate(P->rows_needed, P->rows_formed, P->products,
                                                           P->fold_terms, twopass_fold);
        P->est_owner_ms = est.owner_ms;
        P->est_atomic_ms = est.atomic_ms;
        if (est.atomic_ms < est.owner_ms) {
          // release everything the owner fold built
          for (TileClass& tc : P->tclasses) t.put(tc.tiles);
          P->tclasses.clear();
          for (int** q : {&P->tile_ptr, &P->tile_rows, &P->tile_slot, &P->tile_fptr, &P->tile_fine,
                          &P->off_fptr, &P->off_fine, &P->staged_tiles, &P->halo_ptr, &P->halo_rows,
                          &P->A_pext}) {
            t.put(*q);
            *q = nullptr;
          }
          P->host_fptr.clear();
          P->ntiles = P->TE = P->n_staged = 0;
          P->any_tile_global = false;
          P->cache_bytes = 0;
          spill_need_ints = spill_need_vals = 0;
          atomic = true;
        }
      }
    }
    P->fold_used = atomic ? PTAP_FOLD_ATOMIC : PTAP_FOLD_OWNER;
    if (atomic) {
      // Single-pass forms: rows with |R_I| <= 32, at most 32 entries in P(I,:) and at most 32 in
      // every row of C under them take the short-row kernel; the others the general one, by
      // capacity class.  Rows with an empty P(I,:) or R_I add nothing and are dropped.
      const bool twopass = P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1;
      RowMulArgs gf{};
      gf.nX = gf.nY = n;
      gf.nnzX = P->nnzA;
      gf.nnzY = gf.nnzO = P->nnzP;
      gf.nF = m;
      gf.nnzF = P->nnzC;
      const bool short_ok = !twopass && rowmul_short_fits(gf);
      int* code = t.get<int>(n);
      hipck(launch_rowform_codes(2, n, r, pat.A_rowptr, P->C_rowptr, pat.P_rowptr, pat.P_col, short_ok, code, s));
      int* sorted = nullptr;
      const std::vector<int> hist = classes_from_codes(t, code, nullptr, n, kCodeShort1 + 1, &sorted, s);
      t.put(code);
      P->arows = cap_classes(hist, sorted, lmax);
      long long kept = 0;
      for (int v : hist) kept += v;
      for (int k = 0; k < 2; ++k) {
        P->n_af_short[k] = hist[kCodeShort0 + k];
        P->af_short[k] = group_rows(hist, sorted, kCodeShort0 + k);
      }
      spill_need_ints = spill_ints(P->arows, 1);
      spill_need_vals = spill_need_ints;
      P->rows_formed = (int64_t)kept * (twopass ? 2 : 1);
      t.put(P->pt_ptr);
      t.put(P->pt_row);
      P->pt_ptr = P->pt_row = nullptr;
    }
  }

  // --- Adjoint row classes.  U_I has the distinct columns of the rows of C under P(I,:) as keys
  // (R_I's columns are among them); they are counted on the device.  Rows whose rows of C under
  // P(I,:) hold at most kAdjMaxWalk entries in total go to the short-row kernel.
  if (P->opt.backward) {
    const int lds_max = lmax / 2 >= 64 ? lmax / 2 : 64;
    int* code = t.get<int>(n);
    hipck(launch_adj_codes(pat, r, P->C_rowptr, P->C_col, std::min(kAdjMaxCap, lds_max), code, s));
    int* sorted = nullptr;
    const std::vector<int> hist = classes_from_codes(t, code, nullptr, n, kMaxClassBins, &sorted, s);
    t.put(code);
    // the general kernel holds two tables of this capacity per wavefront
    P->bwd_rows = cap_classes(std::vector<int>(hist.begin(), hist.begin() + 31), sorted, lds_max);
    spill_need_ints = std::max(spill_need_ints, spill_ints(P->bwd_rows, 2));
    spill_need_vals = std::max(spill_need_vals, spill_ints(P->bwd_rows, 2));
    long long off = 0;
    for (int b = 0; b < 32; ++b) off += hist[b];
    for (int b = 32; b < kMaxClassBins; ++b) {
      if (!hist[b]) continue;
      RowClass c;
      c.cap = 1 << (b - 32);
      c.global = c.cap > lds_max;
      c.fast = true;
      c.count = hist[b];
      c.rows = sorted + off;
      off += hist[b];
      P->bwd_rows.push_back(c);
    }
  }
  t.put(r);
  t.put(c_flag);
  t.put(st);
  P->spill_slots = std::max(spill_need_ints, spill_need_vals);
  if (spill_need_ints) P->gtab = t.get<int>(spill_need_ints);
  if (spill_need_vals) P->gval = t.get<double>(spill_need_vals);
  if (P->gtab) hipck(launch_fill_i32(P->gtab, EMPTY, (long long)spill_need_ints, s));
  if (P->gval) hipck(launch_fill_f64(P->gval, 0.0, (long long)spill_need_vals, s));
  hipck(hipStreamSynchronize(s));
}

ptap_status ptap_symbolic(ptap_plan* plan, hipStream_t stream) {
  if (!plan) return PTAP_ERR_INPUT;
  if (plan->sym_done) return PTAP_ERR_STATE;
  // Run on a scratch copy of the plan's state so that a failure leaves the plan unchanged.
  try {
    symbolic_impl(plan, stream);
  } catch (...) {
    const ptap_status st = caught_status();
    // wait for the launches already queued, then release everything the failed phase allocated
    (void)hipStreamSynchronize(stream);
    (void)hipGetLastError();
    plan->mem.release_all();
    ptap_plan fresh;
    fresh.mem.a = plan->mem.a;
    fresh.mem.peak = plan->mem.peak;
    fresh.opt = plan->opt;
    fresh.pat = plan->pat;
    fresh.nnzA = plan->nnzA;
    fresh.nnzP = plan->nnzP;
    fresh.lds_budget = plan->lds_budget;
    fresh.lds_device = plan->lds_device;
    fresh.n_cu = plan->n_cu;
    fresh.owner_waves = plan->owner_waves;
    fresh.lds_hash_max = plan->lds_hash_max;
    fresh.lds_keys_max = plan->lds_keys_max;
    plan->~ptap_plan();
    new (plan) ptap_plan(std::move(fresh));
    return st;
  }
  plan->sym_done = true;
  return PTAP_OK;
}

ptap_status ptap_copy_pattern(const ptap_plan* plan, int32_t* C_rowptr, int32_t* C_col,
                              hipStream_t stream) {
  if (!plan) return PTAP_ERR_INPUT;
  if (!plan->sym_done) return PTAP_ERR_STATE;
  try {
    if (C_rowptr)
      hipck(hipMemcpyAsync(C_rowptr, plan->C_rowptr, ((size_t)plan->pat.m + 1) * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, stream));
    if (C_col && plan->nnzC)
      hipck(hipMemcpyAsync(C_col, plan->C_col, (size_t)plan->nnzC * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, stream));
  } catch (...) {
    return caught_status();
  }
  return PTAP_OK;
}

ptap_status ptap_get_pattern(const ptap_plan* plan, int64_t* nnz_C, const int32_t** C_rowptr,
                             const int32_t** C_col) {
  if (!plan) return PTAP_ERR_INPUT;
  if (!plan->sym_done) return PTAP_ERR_STATE;
  if (nnz_C) *nnz_C = plan->nnzC;
  if (C_rowptr) *C_rowptr = plan->C_rowptr;
  if (C_col) *C_col = plan->C_col;
  return PTAP_OK;
}

static NumericArgs numeric_args(ptap_plan* P, const double* A_val, const double* P_val,
                                double* C_val, int part) {
  NumericArgs a;
  a.p = P->pat;
  a.A_pext = P->A_pext;
  a.A_val = A_val;
  a.P_val = P_val;
  a.C_rowptr = P->C_rowptr;
  a.C_col = P->C_col;
  a.C_val = C_val;
  a.K = P->opt.nblocks;
  a.part = part;
  a.off_fptr = P->off_fptr;
  a.off_fine = P->off_fine;
  a.wide_a = P->wide_a ? 1 : 0;
  a.hash_mul = P->hash_mul;
  return a;
}

// The numeric phase with the device-memory hash tables of the general kernels at gtab / gval
// (the plan's own workspace, or the static scratch of ptap_numeric_noalloc).  Throws Failure.
static void numeric_impl(ptap_plan* P, const double* A_val, const double* P_val, double* C_val,
                         int* gtab, double* gval, hipStream_t s) {
  {
    if (P->nnzC == 0) return;
    if (P->bs > 1) {
      const BsrArgs b{P->pat.A_rowptr, P->pat.A_col, P->pat.P_rowptr, P->pat.P_col, A_val, P_val,
                      P->C_rowptr, P->C_col, C_val, P->pt_ptr, P->pt_row, P->pt_pos};
      if (P->bsr_n_glob) hipck(launch_fill_f64(C_val, 0.0, P->nnzC * P->bs * P->bs, s));
      hipck(launch_bsr_numeric(b, P->bs, P->bsr_rows_lds, P->bsr_n_lds, P->bsr_cap, P->bsr_ncmax, true,
                               P->opt.xcd_remap != 0, s));
      hipck(launch_bsr_numeric(b, P->bs, P->bsr_rows_glob, P->bsr_n_glob, 64, 0, false,
                               P->opt.xcd_remap != 0, s));
      return;
    }
    if (P->opt.algo == PTAP_TWOSTEP) {
      NumericArgs a = numeric_args(P, A_val, P_val, C_val, PART_ALL);
      for (auto& c : P->ap_rows)
        hipck(launch_ap_numeric(a, c, P->AP_rowptr, P->AP_col, P->AP_val, gtab, gval, s));
      const RowMulArgs g1{P->pat.A_rowptr, P->pat.A_col, A_val, P->pat.P_rowptr, P->pat.P_col,
                          P_val, P->AP_rowptr, P->AP_col, P->AP_val, P->pat.n, P->pat.n,
                          P->nnzA, P->nnzP, P->nnzAP};
      for (int k = 0; k < 2; ++k)
        hipck(launch_rowmul_short(g1, P->ap_short[k], P->n_ap_short[k], k == 1, P->n_cu, s));
      hipck(launch_gather(P_val, P->pt_pos, P->PT_val, P->nnzP, s));
      for (auto& c : P->ptc_rows)
        hipck(launch_ptc_numeric(P->pt_ptr, P->pt_row, P->PT_val, P->AP_rowptr, P->AP_col,
                                 P->AP_val, P->C_rowptr, P->C_col, C_val, c, gtab, gval, s));
      const RowMulArgs g2{P->pt_ptr, P->pt_row, P->PT_val, P->AP_rowptr, P->AP_col, P->AP_val,
                          P->C_rowptr, P->C_col, C_val, P->pat.m, P->pat.n,
                          P->nnzP, P->nnzAP, P->nnzC};
      for (int k = 0; k < 2; ++k)
        hipck(launch_rowmul_short(g2, P->ptc_short[k], P->n_ptc_short[k], k == 1, P->n_cu, s));
      return;
    }
    const bool twopass = P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1;
    if (P->fold_used == PTAP_FOLD_ATOMIC) {
      hipck(launch_fill_f64(C_val, 0.0, P->nnzC, s));
      const int parts[2] = {twopass ? PART_OFF : PART_ALL, PART_ON};
      for (int k = 0; k < (twopass ? 2 : 1); ++k) {
        NumericArgs a = numeric_args(P, A_val, P_val, C_val, parts[k]);
        for (auto& c : P->arows) hipck(launch_atomic_numeric(a, c, gtab, gval, s));
      }
      RowMulArgs gf{P->pat.A_rowptr, P->pat.A_col, A_val, P->pat.P_rowptr, P->pat.P_col, P_val,
                    P->pat.P_rowptr, P->pat.P_col, nullptr, P->pat.n, P->pat.n, P->nnzA,
                    P->nnzP, P->nnzP, P_val, P->C_rowptr, P->C_col, C_val, P->pat.m, P->nnzC};
      for (int k = 0; k < 2; ++k)
        hipck(launch_atomic_fold_short(gf, P->af_short[k], P->n_af_short[k], k == 1, P->n_cu, s));
      return;
    }
    if (P->any_tile_global) hipck(launch_fill_f64(C_val, 0.0, P->nnzC, s));
    NumericArgs a = numeric_args(P, A_val, P_val, C_val, twopass ? -1 : PART_ALL);
    if (P->n_staged) {
      const TileSet ts{P->tile_ptr, P->tile_rows, P->tile_slot};
      hipck(launch_staged(a, P->staged_tiles, P->n_staged, ts, P->tile_fptr, P->tile_fine, P->halo_ptr,
                          P->halo_rows, P->staged_L, P->opt.xcd_remap != 0, s));
    }
    for (auto& c : P->tclasses) {
      const TileSet ts{P->tile_ptr, P->tile_rows, P->tile_slot};
      if (c.fast)
        hipck(launch_owner_fast(a, c, ts, P->tile_fptr, P->tile_fine, P->TE, P->owner_waves,
                                P->opt.xcd_remap != 0, s));
      else
        hipck(launch_owner_numeric(a, c, ts, P->tile_fptr, P->tile_fine, P->TE,
                                   P->opt.xcd_remap != 0, gtab, gval, s));
    }
  }
}

ptap_status ptap_numeric(ptap_plan* P, const double* A_val, const double* P_val, double* C_val,
                         hipStream_t s) {
  if (!P) return PTAP_ERR_INPUT;
  if (!P->sym_done) return PTAP_ERR_STATE;
  if ((!A_val && P->nnzA) || (!P_val && P->nnzP) || (!C_val && P->nnzC)) return PTAP_ERR_INPUT;
  try {
    numeric_impl(P, A_val, P_val, C_val, P->gtab, P->gval, s);
  } catch (...) {
    return caught_status();
  }
  return PTAP_OK;
}

// The numeric phase with the general kernels' device-memory hash tables in caller-given memory of
// `slots` keys and values: cleared here by fill kernels (the memory keeps whatever a previous
// call left), then the same launches as ptap_numeric.  Used by ptap_numeric_noalloc.
__attribute__((visibility("hidden"))) ptap_status numeric_with_scratch(
    ptap_plan* P, const double* A_val, const double* P_val, double* C_val, int* keys, double* vals,
    size_t slots, hipStream_t s) {
  if (!P) return PTAP_ERR_INPUT;
  if (!P->sym_done) return PTAP_ERR_STATE;
  if ((!A_val && P->nnzA) || (!P_val && P->nnzP) || (!C_val && P->nnzC)) return PTAP_ERR_INPUT;
  if (P->spill_slots > slots) return PTAP_ERR_TOO_LARGE;
  try {
    if (P->spill_slots) {
      hipck(launch_fill_i32(keys, EMPTY, (long long)P->spill_slots, s));
      hipck(launch_fill_f64(vals, 0.0, (long long)P->spill_slots, s));
    }
    numeric_impl(P, A_val, P_val, C_val, P->spill_slots ? keys : nullptr, P->spill_slots ? vals : nullptr, s);
  } catch (...) {
    return caught_status();
  }
  return PTAP_OK;
}

__attribute__((visibility("hidden"))) size_t plan_scratch_slots(const ptap_plan* P) {
  return P ? P->spill_slots : 0;
}

ptap_status ptap_backward(ptap_plan* P, const double* A_val, const double* P_val,
                          const double* dC_val, double* dA_val, double* dP_val, hipStream_t s) {
  if (!P) return PTAP_ERR_INPUT;
  if (P->bs > 1) return PTAP_ERR_UNSUPPORTED;
  if (!P->sym_done) return PTAP_ERR_STATE;
  if (!P->opt.backward) return PTAP_ERR_STATE;
  if ((!A_val && P->nnzA) || (!P_val && P->nnzP) || (!dC_val && P->nnzC)) return PTAP_ERR_INPUT;
  try {
    if (dA_val) hipck(launch_fill_f64(dA_val, 0.0, P->nnzA, s));
    if (dP_val) hipck(launch_fill_f64(dP_val, 0.0, P->nnzP, s));
    if (!dA_val && !dP_val) return PTAP_OK;
    NumericArgs a = numeric_args(P, A_val, P_val, nullptr, PART_ALL);
    for (auto& c : P->bwd_rows)
      hipck(c.fast ? launch_backward_short(a, dC_val, dA_val, dP_val, c, s)
                   : launch_backward(a, dC_val, dA_val, dP_val, c, P->gtab, P->gval, s));
  } catch (...) {
    const ptap_status st = caught_status();
    return st;
  }
  return PTAP_OK;
}

ptap_status ptap_plan_stats(const ptap_plan* P, ptap_stats* out) {
  if (!P || !out) return PTAP_ERR_INPUT;
  memset(out, 0, sizeof(*out));
  out->nnz_C = P->nnzC;
  out->nnz_AP = P->nnzAP;
  out->workspace_bytes = P->mem.current;
  out->peak_bytes = P->mem.peak;
  out->pattern_bytes = P->pattern_bytes;
  out->rows_formed = P->rows_formed;
  out->rows_needed = P->rows_needed;
  out->fold_terms = P->fold_terms;
  out->n_tiles = P->ntiles;
  out->fold_used = P->fold_used;
  out->algo = P->opt.algo;
  out->nblocks = P->opt.nblocks;
  out->cache_bytes = P->cache_bytes;
  out->block_size = P->bs;
  out->staged_tiles = P->n_staged;
  out->staged_lds_bytes = P->n_staged ? P->staged_L.total : 0;
  out->table_slots = (int64_t)P->spill_slots;
  out->tile_entries = P->ntiles ? P->TE : 0;
  out->est_owner_ms = P->est_owner_ms;
  out->est_atomic_ms = P->est_atomic_ms;
  out->hash_mul = P->ntiles > 0 ? (int64_t)P->hash_mul : 0;
  return PTAP_OK;
}

void ptap_plan_destroy(ptap_plan* P) {
  if (!P) return;
  P->mem.release_all();
  delete P;
}

ptap_status ptap_batch_create(ptap_batch** out, ptap_plan* const* plans, const int32_t* level,
                              int32_t count, const ptap_allocator* alloc, hipStream_t stream) {
  if (!out) return PTAP_ERR_INPUT;
  *out = nullptr;
  if (count < 1 || !plans) return PTAP_ERR_INPUT;
  if (alloc && (!alloc->alloc || !alloc->release)) return PTAP_ERR_INPUT;
  for (int k = 0; k < count; ++k) {
    if (!plans[k]) return PTAP_ERR_INPUT;
    if (plans[k]->bs > 1) return PTAP_ERR_UNSUPPORTED;
    if (!plans[k]->sym_done) return PTAP_ERR_STATE;
    if (plans[k]->opt.algo == PTAP_TWOSTEP) return PTAP_ERR_UNSUPPORTED;
  }
  ptap_batch* b = new (std::nothrow) ptap_batch();
  if (!b) return PTAP_ERR_OOM;
  if (alloc) b->mem.a = *alloc;
  try {
    b->plans.assign(plans, plans + count);
    b->level.resize(count);
    for (int k = 0; k < count; ++k) b->level[k] = level ? level[k] : 0;
    b->levels = b->level;
    std::sort(b->levels.begin(), b->levels.end());
    b->levels.erase(std::unique(b->levels.begin(), b->levels.end()), b->levels.end());
    const int L = (int)b->levels.size();
    b->level_plans.resize(L);
    for (int k = 0; k < count; ++k) {
      const int l = (int)(std::lower_bound(b->levels.begin(), b->levels.end(), b->level[k]) - b->levels.begin());
      b->level_plans[l].push_back(k);
    }
    // work lists: the short-row tiles of every plan of a level, plan by plan, tiles in order
    for (int l = 0; l < L; ++l) {
      std::vector<std::pair<int, int2>> w;
      for (int k : b->level_plans[l]) {
        const ptap_plan* P = plans[k];
        if (P->wide_a) continue;  // launched on its own (the batched kernel reads A by offset)
        for (const TileClass& c : P->tclasses) {
          if (!c.fast) continue;
          for (int tl : c.host_tiles)
            w.push_back({P->host_fptr[tl + 1] - P->host_fptr[tl], make_int2(k, tl)});
        }
        b->lds = std::max(b->lds, owner_fast_lds_bytes(P->TE, kFastWaves));
      }
      std::vector<int2> items(w.size());
      for (size_t q = 0; q < w.size(); ++q) items[q] = w[q].second;
      int2* d = b->mem.get<int2>(items.size());
      if (!items.empty()) {
        hipck(hipMemcpyAsync(d, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, stream));
        hipck(hipStreamSynchronize(stream));
      }
      b->items.push_back(d);
      b->nitems.push_back((int)items.size());
    }
    b->counters = b->mem.get<int>((size_t)L * kXcds);
    b->d_plans = b->mem.get<OwnerBatchPlan>(count);
    int dev = 0, cus = 0;
    hipck(hipGetDevice(&dev));
    hipck(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->grid = std::max(1, cus * 2);
    hipck(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  } catch (...) {
    const ptap_status st = caught_status();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->mem.release_all();
    delete b;
    return st;
  }
  *out = b;
  return PTAP_OK;
}

static void batch_record(ptap_batch* b, hipStream_t s) {
  const int count = (int)b->plans.size();
  std::vector<OwnerBatchPlan> desc(count);
  for (int k = 0; k < count; ++k) {
    ptap_plan* P = b->plans[k];
    NumericArgs a = numeric_args(P, b->A_vals[k], b->P_vals[k], b->C_vals[k],
                                 (P->opt.algo == PTAP_ALLATONCE && P->opt.nblocks > 1) ? -1 : PART_ALL);
    desc[k] = OwnerBatchPlan{a, TileSet{P->tile_ptr, P->tile_rows, P->tile_slot}, P->tile_fptr,
                             P->tile_fine, P->TE};
  }
  hipck(hipMemcpyAsync(b->d_plans, desc.data(), desc.size() * sizeof(OwnerBatchPlan),
                       hipMemcpyHostToDevice, s));
  hipck(hipStreamSynchronize(s));
  hipck(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  hipError_t err = hipSuccess;
  for (size_t l = 0; l < b->levels.size() && err == hipSuccess; ++l) {
    // the work counters of the level's persistent launch; levels of one plan have none (on the
    // 64^3 hierarchy the graph took 4.5% longer than plain launches with a fill at every level,
    // 1.1% without)
    const bool persistent = b->level_plans[l].size() > 1 && b->nitems[l] > 0;
    if (persistent) err = launch_fill_i32(b->counters + l * kXcds, 0, kXcds, b->cap);
    for (int k : b->level_plans[l]) {
      ptap_plan* P = b->plans[k];
      const NumericArgs& a = desc[k].a;
      if (err == hipSuccess && P->any_tile_global) err = launch_fill_f64(b->C_vals[k], 0.0, P->nnzC, b->cap);
      // one plan at this level, or A's values past 2 GiB: the plan's own launch (its grid, tiles
      // mapped to XCDs in order).  The persistent work-list kernel was slower for single-plan
      // levels: 9.07 against 7.00 ms on the 256^3 six-level hierarchy, 0.47 against 0.24 ms on
      // 64^3 down to 2^3 (its 512 workgroups per level mostly find no work on small levels).
      const bool single = b->level_plans[l].size() == 1 || P->wide_a;
      if (P->fold_used == PTAP_FOLD_ATOMIC) {  // the atomic fold: the plan's own launches
        if (err == hipSuccess) {
          try {
            numeric_impl(P, b->A_vals[k], b->P_vals[k], b->C_vals[k], P->gtab, P->gval, b->cap);
          } catch (...) {
            err = hipErrorUnknown;
          }
        }
        continue;
      }
      if (err == hipSuccess && P->n_staged)  // staged tiles: the plan's own launch
        err = launch_staged(a, P->staged_tiles, P->n_staged, TileSet{P->tile_ptr, P->tile_rows, P->tile_slot},
                            P->tile_fptr, P->tile_fine, P->halo_ptr, P->halo_rows, P->staged_L,
                            P->opt.xcd_remap != 0, b->cap);
      for (const TileClass& c : P->tclasses) {
        if (err != hipSuccess) break;
        const TileSet ts{P->tile_ptr, P->tile_rows, P->tile_slot};
        if (!c.fast)
          err = launch_owner_numeric(a, c, ts, P->tile_fptr, P->tile_fine, P->TE,
                                     P->opt.xcd_remap != 0, P->gtab, P->gval, b->cap);
        else if (single)
          err = launch_owner_fast(a, c, ts, P->tile_fptr, P->tile_fine, P->TE, P->owner_waves,
                                  P->opt.xcd_remap != 0, b->cap);
      }
    }
    // the short-row tiles of a level's several plans in one persistent launch
    if (err == hipSuccess && persistent)
      err = launch_owner_fast_batch(b->d_plans, b->items[l], b->nitems[l], b->counters + l * kXcds,
                                    b->grid, b->lds, b->cap);
  }
  hipGraph_t g = nullptr;
  const hipError_t end = hipStreamEndCapture(b->cap, &g);
  hipck(err);
  hipck(end);
  b->graph = g;
  hipck(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
}

ptap_status ptap_batch_numeric(ptap_batch* b, const double* const* A_vals,
                               const double* const* P_vals, double* const* C_vals,
                               hipStream_t stream) {
  if (!b || !A_vals || !P_vals || !C_vals) return PTAP_ERR_INPUT;
  const int count = (int)b->plans.size();
  for (int k = 0; k < count; ++k) {
    const ptap_plan* P = b->plans[k];
    if ((!A_vals[k] && P->nnzA) || (!P_vals[k] && P->nnzP) || (!C_vals[k] && P->nnzC))
      return PTAP_ERR_INPUT;
  }
  try {
    if (!b->exec) {
      b->A_vals.assign(A_vals, A_vals + count);
      b->P_vals.assign(P_vals, P_vals + count);
      b->C_vals.assign(C_vals, C_vals + count);
      batch_record(b, stream);
    } else {
      for (int k = 0; k < count; ++k)
        if (A_vals[k] != b->A_vals[k] || P_vals[k] != b->P_vals[k] || C_vals[k] != b->C_vals[k])
          return PTAP_ERR_INPUT;
    }
    hipck(hipGraphLaunch(b->exec, stream));
  } catch (...) {
    const ptap_status st = caught_status();
    return st;
  }
  return PTAP_OK;
}

void ptap_batch_destroy(ptap_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) {
    (void)hipStreamSynchronize(b->cap);
    (void)hipStreamDestroy(b->cap);
  }
  b->mem.release_all();
  delete b;
}

}  // extern "C"
