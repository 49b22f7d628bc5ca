// Building blocks of the short-row kernels (two rows per wavefront, one per 32-lane half):
// raw buffer loads, half-wavefront scans, one step of the flattened product walk, and the
// 64-slot LDS hash table of a row with at most 32 keys.  Used by the owner fold (owner.hip) and
// by the row-times-matrix products of the two-step method (rowmul.hip).
#pragma once

#include "device.hpp"

namespace ptapk {

constexpr int kHalf = 32;
constexpr int kCap = 64;  // slots of one row's table (at most 32 keys, load <= 1/2)
constexpr int kCapShift = 32 - 6;

// Record of one nonempty segment of a flattened product walk (one entry X(r,k) of the outer
// row): its weight and the offset that turns a product number q of the row into the index
// q + base of the inner matrix's entry.  The owner fold reuses the record area for its owned
// entries (weight P(I,i), start (base) and end (pad) of row i of the tile).
struct SegRec {
  double w;
  int base;
  int pad;
};

// Per-wavefront LDS scratch: a table and a record list for each half.
struct HalfScratch {
  int keys[2][kCap];
  double vals[2][kCap];
  SegRec rec[2][kHalf];
};

// Raw buffer resources: 32-bit byte offsets instead of 64-bit addresses, one 8-byte load for a
// pair of row pointers, and reads past the end of an array return 0 instead of faulting.  The
// texture address unit handles a 4-byte load at 16 lanes per cycle but an 8-byte one at 4 lanes
// per cycle even when the lanes share an address, so values needed by a whole half-wavefront
// (a row's index and extents) are loaded by one lane and broadcast with readlane.
typedef unsigned v2u __attribute__((ext_vector_type(2)));
constexpr int kRawBufferFlags = 0x00020000;  // 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRawBufferFlags);
}
__device__ __forceinline__ v2u ld_pair(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, idx * 4, 0, 0);
}

// Inclusive prefix sum (or prefix OR) over each 32-lane half of the wavefront, in VALU only:
// DPP row shifts by 1, 2, 4, 8 scan each 16-lane row, then lane 15 of rows 0 and 2 is broadcast
// into rows 1 and 3.  Lanes whose source lies outside the row keep the identity (old = 0).
// Every lane of the wavefront must be active.
__device__ __forceinline__ int half_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
  return v;
}
__device__ __forceinline__ int half_or_scan(int v) {
  v |= __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);
  v |= __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);
  v |= __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
  v |= __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
  v |= __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
  return v;
}

__device__ __forceinline__ int ld_col(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0);
}
__device__ __forceinline__ double ld_dbl(__amdgpu_buffer_rsrc_t r, int idx) {
  const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
__device__ __forceinline__ int ld_i32(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0);
}

// The value of lane 31 (half 0) or lane 63 (half 1): the half's total after a scan.
__device__ __forceinline__ int half_total(int v, int half) {
  const int t0 = __builtin_amdgcn_readlane(v, 31), t1 = __builtin_amdgcn_readlane(v, 63);
  return half ? t1 : t0;
}

// One step of the flattened product walk of a half: product k = 32 st + sub of the row (if it
// exists) is entry k + base of P, weighted by A(I,J) of its segment.  `before` counts the
// nonempty segments ending at or before the step's window and is advanced past it.
struct ProdLoad {
  int j;     // column of P's entry (0 where there is no product)
  double v;  // value of P's entry
  double w;  // A(I,J)
  bool ok;   // the product exists (tested only where it is inserted, so that the loads of
             // several steps stay in flight together)
};
__device__ __forceinline__ ProdLoad prod_load(int st, int incl, int len, int Th, int sub, int half,
                                              int& before, const SegRec* rec,
                                              __amdgpu_buffer_rsrc_t rPc, __amdgpu_buffer_rsrc_t rPv) {
  const int k0 = st * kHalf;
  const int d = incl - k0 - 1;
  const int bit = (len > 0 && (unsigned)d < (unsigned)kHalf) ? (int)(1u << d) : 0;
  const unsigned ends = (unsigned)half_total(half_or_scan(bit), half);
  const int k = k0 + sub;
  const int rk = (before + __popc(ends & ((1u << sub) - 1u))) & (kHalf - 1);
  const SegRec rc = rec[rk];
  const int e = k < Th ? k + rc.base : -1;
  ProdLoad r{ld_col(rPc, e), ld_dbl(rPv, e), rc.w, k < Th};
  before += __popc(ends);
  return r;
}

// Default multiplier of the 64-slot tables' hash (the top 6 bits of key * mul): the golden
// ratio times 2^32.  The owner fold's short-row kernel takes a multiplier chosen per plan instead.
constexpr unsigned kHashMul = 0x9E3779B1u;

// R_I(key) += v in a 64-slot LDS table.  A plain read finds keys already present (most of a
// row's products hit a key inserted before), so only first insertions use compare-and-swap.
// The probe is bounded by the table size (a half never holds more than 32 keys, so the bound is
// never reached).  Any odd multiplier gives the same result; it only moves keys between slots.
__device__ __forceinline__ void hash_add64(int* keys, double* vals, int key, double v,
                                           unsigned mul = kHashMul) {
  unsigned s = ((unsigned)key * mul) >> kCapShift;
#pragma unroll 1  // rarely more than one probe: unrolling only adds exec-mask bookkeeping
  for (int it = 0; it < kCap; ++it) {
    int seen = keys[s];
    if (seen == EMPTY) seen = atomicCAS(keys + s, EMPTY, key);
    if (seen == EMPTY || seen == key) {
      atomicAdd(vals + s, v);
      return;
    }
    s = (s + 1) & (kCap - 1);
  }
}


// Slot of key in a row's 64-slot table, or -1 (the table's inserts are complete).  Rolled: the
// first read settles nearly every lookup.
__device__ __forceinline__ int hash_find64(const int* keys, int key, unsigned mul = kHashMul) {
  unsigned s = ((unsigned)key * mul) >> kCapShift;
  int kf = keys[s];
#pragma unroll 1
  for (int it = 1; kf != key && kf != EMPTY && it < kCap; ++it) {
    s = (s + 1) & (kCap - 1);
    kf = keys[s];
  }
  return kf == key ? (int)s : -1;
}

}  // namespace ptapk
