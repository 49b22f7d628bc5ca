// Host-side plan structure and kernel launch wrappers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/ptap.h"
#include "device.hpp"

namespace ptapk {

// A set of rows processed by one launch: all rows whose hash table has `cap` slots, held in
// LDS (global = false) or in device memory (global = true).
struct RowClass {
  int cap = 0;
  bool global = false;
  bool fast = false;  // adjoint: short-row kernel (adjoint.hip)
  int count = 0;
  int* rows = nullptr;  // device, `count` row indices in ascending order
};

// Device arrays of the inputs' patterns (caller-owned).
struct Patterns {
  int n, m;
  const int* A_rowptr;
  const int* A_col;
  const int* P_rowptr;
  const int* P_col;
};

// Owner-fold launch group: tiles sharing a hash-table capacity and tile placement.
struct TileClass {
  int cap = 0;
  bool hash_global = false;
  bool tile_global = false;
  bool fast = false;     // short-row kernel (owner.hip)
  bool long_c = false;   // short-row kernel: some row of C in these tiles has more than 64 columns
  int count = 0;
  int* tiles = nullptr;  // device, tile ids
  std::vector<int> host_tiles;
};

// Limits of on-chip storage per launch (bytes of LDS per workgroup are set per kernel).
constexpr int kWavesPerBlock = 4;
constexpr int kLdsHashMax = 1024;       // largest LDS table (slots) of a numeric kernel
constexpr int kLdsKeysMax = 2048;       // largest LDS key-only table (slots) of a symbolic kernel
constexpr int kDefaultTileEntries = 4096;  // general kernel
constexpr int kTileLdsTarget = 81920;     // bytes of LDS per owner workgroup (two per CU)
constexpr int kSpillWaves = 512;        // concurrent wavefronts of a spill (global-table) launch
constexpr int kXcds = 8;                // accelerator complex dies of the MI355X

// ---------------------------------------------------------------------------------------
// Launch wrappers (kernels.hip).  All take a stream and return hipError_t.
// ---------------------------------------------------------------------------------------
hipError_t launch_fill_i32(int* p, int value, long long count, hipStream_t s);
hipError_t launch_fill_f64(double* p, double value, long long count, hipStream_t s);
hipError_t launch_stream_sum(const double* x, long long n, double* out, hipStream_t s);
hipError_t launch_count_cols(const int* col, long long nnz, int* cnt, hipStream_t s);
hipError_t launch_transpose_fill(const int* rowptr, const int* col, int nrows, int* cursor,
                                 int* t_row, int* t_pos, hipStream_t s);
// out[0..4]: needed rows, fold terms, max |R_I|, max(nnz(P(I,:)), nnz(A(I,:))), products
// A(I,J) P(J,j) of the needed rows (the sum of w over them); out zeroed by the caller
hipError_t launch_row_stats(const Patterns& p, const int* r, const int* w, unsigned long long* out,
                            hipStream_t s);
hipError_t launch_ap_row_count(const Patterns& p, const RowClass& rc, int* r_out, int* gtab,
                               hipStream_t s);
hipError_t launch_ap_row_fill(const Patterns& p, const RowClass& rc, const int* AP_rowptr,
                              int* AP_col, int* gtab, hipStream_t s);
hipError_t launch_c_bound(const int* pt_ptr, const int* pt_row, const int* r, int m,
                          long long* bound, hipStream_t s);
// C pattern by the row form: all-at-once (recompute S(R_I)) or two-step (read stored AP rows).
hipError_t launch_c_rows(const Patterns& p, const int* pt_ptr, const int* pt_row,
                         const int* AP_rowptr, const int* AP_col, const RowClass& rc, bool fill,
                         int* cnt_out, const int* C_rowptr, int* C_col, int* gtab, hipStream_t s);
// Count pass: cnt_out[t] = number of distinct fine rows of tile t; rmax_out[2t] = max |R_I| and
// rmax_out[2t+1] = max row length of A and of P over them.  Fill pass: the sorted rows.  Only
// entries P(I,i) that part (PART_ALL, PART_OFF, PART_ON with K blocks) takes make I a row of t.
hipError_t launch_tile_fine(const Patterns& p, const int* pt_ptr, const int* pt_row,
                            const TileSet& ts, int ntiles, const int* r, bool fill, int* cnt_out,
                            int* rmax_out, const int* fptr, int* fine, int part, int K,
                            hipStream_t s);
// Reorder the lists of the given tiles (in place) by the count of the row's entries of P the
// tile owns.
hipError_t launch_tile_order(const Patterns& p, const int* tiles, int ntiles, const int* fptr,
                             int* fine, const int* slot, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Device symbolic building blocks (symbolic.hip).
// ---------------------------------------------------------------------------------------
// Exclusive prefix sum of n int counts into out[0..n] (out[n] = total; out may alias in).
// scratch: scan_scratch_count(n) int64 values, the last of which receives the total; *flag |= 1
// if the total exceeds INT32_MAX.
size_t scan_scratch_count(long long n);
hipError_t launch_scan_i32(const int* in, long long n, int* out, long long* scratch, int* flag,
                           hipStream_t s);
// Row classes by a stable counting sort over codes in [0, nbins) (negative: dropped); item k is
// row list[k] (or k).  sorted: count ints; hist: nbins ints (group sizes, groups in code order);
// scratch: class_scratch_ints(count, nbins) ints; scan_scratch as for launch_scan_i32 over
// nbins * ceil(count / 256) cells.
constexpr int kMaxClassBins = 64;
constexpr int kCodeShort0 = 31;  // row-form short lists (rows of X with <= kHalfLanes entries)
constexpr int kCodeShort1 = 32;  // (longer rows of X)
size_t class_scratch_ints(int count, int nbins);
hipError_t launch_class_build(const int* code, const int* list, int count, int nbins, int* scratch,
                              long long* scan_scratch, int* flag, int* sorted, int* hist, hipStream_t s);
// code[k] = log2 of the hash capacity for need[list[k]] keys (list null: need[k]), -1 if <= 0.
hipError_t launch_cap_codes_i32(const int* need, const int* list, int count, int* code, hipStream_t s);
hipError_t launch_cap_codes_i64(const long long* need, const int* list, int count, int* code, hipStream_t s);
// Pattern checks; err and cnt[0..1] zeroed by the caller.  Valid iff err == 0 and cnt[0] == cnt[1].
hipError_t launch_validate_pattern(const int* rowptr, const int* col, int nrows, int ncols, long long nnz,
                                   int* err, unsigned long long* cnt, hipStream_t s);
// |R_I| and min(w_I, m) of every fine row; rows whose product count could overflow the one-pass
// table get r = 0 and are appended to ovf (*novf zeroed by the caller).
hipError_t launch_ap_count(const Patterns& p, int* r, int* w, int* ovf, int* novf, hipStream_t s);
// C's pattern by the two-level union over rows [row0, row1): count pass (cnt; flag 1 and ovf /
// novf for rows left to the class launches; flag 2 for rows written sorted to the row store,
// kRowStore ints per row of C, when store is given; flag 0 and *nfill += 1 for the others) or
// fill pass (rows of flag 0).  launch_c_from_store copies the stored rows into C_col.
constexpr int kRowStore = 32;
hipError_t launch_c_two_level(const Patterns& p, const int* pt_ptr, const int* pt_row, bool fill, int* cnt,
                              unsigned char* flag, int* ovf, int* novf, const int* C_rowptr, int* C_col,
                              int* store, int* nfill, int row0, int row1, hipStream_t s);
hipError_t launch_c_from_store(const int* C_rowptr, const int* store, const unsigned char* flag, int row0, int row1,
                               int* C_col, hipStream_t s);
hipError_t launch_c_bound_list(const int* pt_ptr, const int* pt_row, const int* r, const int* list, int count,
                               int m, long long* bound, hipStream_t s);
hipError_t launch_tile_slot(const int* tptr, const int* trows, int ntiles, int* slot, hipStream_t s);
// out[0] = max over rows with P(I,:) non-empty of min over i in P(I,:) of |C(i,:)| (a bound on
// |R_I|), out[1] = max over rows of max(nnz(P(I,:)), nnz(A(I,:))); out zeroed by the caller.
hipError_t launch_row_bounds(const Patterns& p, const int* C_rowptr, unsigned* out, hipStream_t s);
// Adjoint launch classes: code[I] = log2 of the table capacity (general kernel), 32 + that
// (short-row kernel: tables of at most fast_cap slots), or -1 (empty P(I,:)).
hipError_t launch_adj_codes(const Patterns& p, const int* r, const int* C_rowptr, const int* C_col, int fast_cap,
                            int* code, hipStream_t s);
// Launch-class codes of the row-form kernels; mode 0: rows of AP, 1: rows of C, 2: atomic fold.
hipError_t launch_rowform_codes(int mode, int nrows, const int* r, const int* x_ptr, const int* c_ptr,
                                const int* P_rowptr, const int* P_col, bool short_ok, int* code, hipStream_t s);

struct NumericArgs {
  Patterns p;
  const int* A_pext;  // numeric cache, or null: per entry A(I,J), (start of P(J,:) << 6) | |P(J,:)|
  const double* A_val;
  const double* P_val;
  const int* C_rowptr;
  const int* C_col;
  double* C_val;
  int K;
  int part;  // FoldPart
  // two-pass all-at-once: per tile, the fine rows with off-block entries owned by the tile (the
  // first pass walks only these); null otherwise
  const int* off_fptr;
  const int* off_fine;
  // A's values span 2 GiB or more (nnz(A) >= 2^28): the short-row owner kernel reads them by
  // 64-bit address instead of a 32-bit buffer offset
  int wide_a;
  // multiplier of the short-row owner kernel's R_I hash (odd; chosen per plan at symbolic time)
  unsigned hash_mul;
};
hipError_t launch_pext(const Patterns& p, long long nnzA, int* out, hipStream_t s);

// Block-sparse (BSR) numeric in the row form: one workgroup per row of C (bsr.hip).
struct BsrArgs {
  const int* A_rowptr;
  const int* A_col;
  const int* P_rowptr;
  const int* P_col;
  const double* A_val;  // nnz(A) blocks of bs*bs, row-major
  const double* P_val;
  const int* C_rowptr;
  const int* C_col;
  double* C_val;
  const int* pt_ptr;  // column lists of P: fine rows and positions of the blocks P(I,i)
  const int* pt_row;
  const int* pt_pos;
};
constexpr int kBsrMaxBlock = 8;
size_t bsr_lds_bytes(int bs, int cap, int ncmax, bool lds_acc);
hipError_t launch_bsr_numeric(const BsrArgs& a, int bs, const int* rows, int nrows, int cap, int ncmax,
                              bool lds_acc, bool remap, hipStream_t s);
hipError_t launch_atomic_numeric(const NumericArgs& a, const RowClass& rc, int* gtab, double* gval,
                                 hipStream_t s);
size_t owner_general_lds_bytes(int TE, int cap, bool hash_global, bool tile_global);
hipError_t launch_owner_numeric(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                                const int* tile_fptr, const int* tile_fine, int tile_entries,
                                bool xcd_remap, int* gtab, double* gval, hipStream_t s);
// Short-row owner kernel (owner.hip): tiles whose fine rows have |R_I| <= 32 and at most 32
// entries in their rows of A and of P.
constexpr int kFastMaxKeys = 32;
constexpr int kFastWaves = 16;
size_t owner_fast_wave_bytes();
size_t owner_fast_lds_bytes(int TE, int nw);
hipError_t launch_owner_fast(const NumericArgs& a, const TileClass& tc, const TileSet& ts,
                             const int* tile_fptr, const int* tile_fine, int TE, int nw,
                             bool xcd_remap, hipStream_t s);
// Staged-tile owner kernel (staged.hip): a tile's halo rows of P are copied into LDS and R_I is
// held in the positions of one of the tile's rows of C.  Tiles qualify when their fine rows have
// at most kStagedMaxA entries in A(I,:) and kStagedMaxP in P(I,:), their rows of C at most
// kStagedMaxRank entries, and the LDS layout of the launch fits the device.
constexpr int kStagedWaves = 8;
constexpr int kStagedMaxA = 28;
constexpr int kStagedMaxP = 8;
constexpr int kStagedMaxRank = 32;
constexpr int kStagedMaxHalo = 4096;  // halo rows the symbolic pass can list per tile
constexpr int kStagedMaxCols = 2048;  // distinct coarse columns it can count per tile
constexpr int kStagedMaxRows = 1024;  // owned rows per tile (positions fit the 16-bit tables)
constexpr int kStagedTileEntries = 1728;  // default tile size (entries of C) when staging

struct StagedCaps {  // maxima over the tiles of one launch
  int NR;  // owned rows of C
  int TE;  // entries of those rows
  int NH;  // halo rows
  int SE;  // entries of P in the halo rows
  int UL;  // distinct coarse columns among them
};
struct StagedLayout {  // dynamic LDS of one launch: capacities and byte offsets
  int NR, TE, NH, SE, ULp, JHlog, UHlog;
  int o_sval, o_tv, o_R, o_rec, o_jh, o_scol, o_tcl, o_trp, o_tcs, o_own, o_M, total;
};

inline int host_log2_ceil(long long v) {
  int b = 0;
  while ((1LL << b) < v) ++b;
  return b;
}

// LDS bytes of a staged launch with these caps and nw wavefronts (and the layout, if L is given).
inline size_t staged_layout(const StagedCaps& c, int nw, StagedLayout* L) {
  StagedLayout l{};
  l.NR = c.NR;
  l.TE = c.TE;
  l.NH = c.NH;
  l.SE = c.SE;
  l.ULp = (c.UL + 3) & ~3;
  l.JHlog = host_log2_ceil(std::max(64, c.NH + c.NH / 2));
  l.UHlog = host_log2_ceil(std::max(64, 2 * c.UL));
  auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
  size_t o = 0;
  l.o_sval = (int)o;
  o = al(o + (size_t)c.SE * 8);
  l.o_tv = (int)o;
  o = al(o + (size_t)c.TE * 8);
  l.o_R = (int)o;
  // R: 16 rows per wavefront of kStagedMaxRank + 1 doubles; the set-up temporaries share it
  // fold records (16 bytes; at most 2 per lane) follow R
  const size_t rbytes = (size_t)nw * (WAVE / 4) * (kStagedMaxRank + 1) * 8;
  const size_t recbytes = (size_t)nw * 2 * WAVE * 16;
  const size_t tbytes = (((size_t)2 << l.UHlog) + 3 * (size_t)c.NH + 1 + (size_t)c.SE + (size_t)c.NR) * 4 +
                        (size_t)c.TE * 2;
  l.o_rec = (int)(o + rbytes);
  o = al(o + std::max(rbytes + recbytes, tbytes));
  l.o_jh = (int)o;
  o = al(o + ((size_t)8 << l.JHlog));
  l.o_scol = (int)o;
  o = al(o + (size_t)c.SE * 2);
  l.o_tcl = (int)o;
  o = al(o + (size_t)c.TE * 2);
  l.o_trp = (int)o;
  o = al(o + ((size_t)c.NR + 1) * 4);
  l.o_tcs = (int)o;
  o = al(o + (size_t)c.NR * 4);
  l.o_own = (int)o;
  o = al(o + (size_t)l.ULp * 2);
  l.o_M = (int)o;
  o = al(o + (size_t)c.NR * l.ULp);
  l.total = (int)o;
  if (L) *L = l;
  return o;
}
// Count pass (fill = false): stats[6t..6t+5] for every listed tile t (halo rows, their entries of
// P, distinct coarse columns, longest row of A and of P over the fine rows, table overflow).
// Fill pass: the sorted halo rows of the listed tiles into halo_rows at halo_ptr[t].
hipError_t launch_tile_halo(const Patterns& p, const int* tiles, int ntiles, const int* tile_fptr,
                            const int* tile_fine, bool fill, int* stats, const int* halo_ptr,
                            int* halo_rows, hipStream_t s);
hipError_t launch_staged(const NumericArgs& a, const int* tiles, int ntiles, const TileSet& ts,
                         const int* tile_fptr, const int* tile_fine, const int* halo_ptr,
                         const int* halo_rows, const StagedLayout& L, bool xcd_remap, hipStream_t s);

// Batched owner fold: a device-side description of one plan (values included).
struct OwnerBatchPlan {
  NumericArgs a;
  TileSet ts;
  const int* tile_fptr;
  const int* tile_fine;
  int TE;
};
// counters: kXcds work counters, zeroed before the launch
hipError_t launch_owner_fast_batch(const OwnerBatchPlan* plans, const int2* items, int nitems,
                                   int* counters, int grid, size_t lds, hipStream_t s);
// Two-step numeric pieces.
hipError_t launch_ap_numeric(const NumericArgs& a, const RowClass& rc, const int* AP_rowptr,
                             const int* AP_col, double* AP_val, int* gtab, double* gval,
                             hipStream_t s);
hipError_t launch_gather(const double* src, const int* idx, double* dst, long long count,
                         hipStream_t s);
// Short-row form of both two-step products (rowmul.hip): O(r,:) = sum_k X(r,k) Y(k,:) into O's
// stored pattern, for rows with at most 32 entries in O(r,:); long_x: the rows listed may have
// more than 32 entries in X(r,:).  O has nX rows.
struct RowMulArgs {
  const int* X_rowptr;
  const int* X_col;
  const double* X_val;
  const int* Y_rowptr;
  const int* Y_col;
  const double* Y_val;
  const int* O_rowptr;
  const int* O_col;
  double* O_val;
  int nX, nY;
  long long nnzX, nnzY, nnzO;
  // atomic fold only: O_rowptr / O_col are P's (the entries P(I,i) folded), F_val P's values,
  // and C += P(I,:) (x) R_I goes into F_out on C's pattern (F_rowptr, F_col; nF rows, nnzF entries)
  const double* F_val;
  const int* F_rowptr;
  const int* F_col;
  double* F_out;
  int nF;
  long long nnzF;
};
constexpr int kRowMulMaxLen = 32;
constexpr int kHalfLanes = 32;  // entries of X(r,:) one pass of the short-row walk takes
bool rowmul_short_fits(const RowMulArgs& g);  // byte extents within the 32-bit buffer range
hipError_t launch_rowmul_short(const RowMulArgs& g, const int* rows, int count, bool long_x,
                               int n_cu, hipStream_t s);
// Short-row atomic fold (F1): X = A, Y = P; rows I with |R_I| <= 32, at most 32 entries in
// P(I,:) and at most 32 in each row of C under them.  C must be zeroed first.
hipError_t launch_atomic_fold_short(const RowMulArgs& g, const int* rows, int count, bool long_x,
                                    int n_cu, hipStream_t s);
hipError_t launch_ptc_numeric(const int* pt_ptr, const int* pt_row, const double* PT_val,
                              const int* AP_rowptr, const int* AP_col, const double* AP_val,
                              const int* C_rowptr, const int* C_col, double* C_val,
                              const RowClass& rc, int* gtab, double* gval, hipStream_t s);
// Adjoint.
hipError_t launch_backward(const NumericArgs& a, const double* dC, double* dA, double* dP,
                           const RowClass& rc, int* gtab, double* gval, hipStream_t s);
// Short-row adjoint (adjoint.hip): rows with 1..kAdjMaxSegs entries in P(I,:), at most
// kAdjMaxWalk entries in the rows of dC under them, and a table of at most kAdjMaxCap slots.
constexpr int kAdjPasses = 4;
constexpr int kAdjMaxWalk = kAdjPasses * WAVE;
constexpr int kAdjMaxSegs = WAVE;
constexpr int kAdjMaxCap = 512;
size_t backward_short_lds_bytes(int cap);
hipError_t launch_backward_short(const NumericArgs& a, const double* dC, double* dA, double* dP,
                                 const RowClass& rc, hipStream_t s);

}  // namespace ptapk
