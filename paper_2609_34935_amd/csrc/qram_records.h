// Record helpers of the qubit encoding's shared tier-2 site lists.  They are
// __host__ __device__ so that their handling of damaged records can be
// exercised by a host program (tests/records_check.cpp).
//
// Record of one class (uint16 words, `rec` per record): [0] address entries,
// [1] bus mask | tagged tokens << 8, [2 .. 2+lmax) address entries,
// [2 + lmax + t] site of tagged token t (EMPTY: on the bus or lost),
// [2 + lmax + k] the split set D of the address (kept in every class slot).
// A count read back from a record is trusted only up to lmax: a larger one
// cannot come from a correct step, raises ERR_LIST and is clamped, so the
// copy loops never run past a record.
#pragma once

#include "qram_internal.h"

#define QR_HD __host__ __device__ __forceinline__

namespace qr {

constexpr uint32_t REC_EMPTY = 0xFFFFu;

// Index of the lowest set bit of m (m != 0).
QR_HD uint32_t low_bit(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

QR_HD void flag_err(uint32_t *err, uint32_t bits) {
#ifdef __HIP_DEVICE_COMPILE__
  atomicOr(err, bits);
#else
  *err |= bits;
#endif
}

// A list count read from memory, bounded by the list capacity lmax.
QR_HD uint32_t rec_count(uint32_t cnt, int lmax, uint32_t *err) {
  if (cnt <= (uint32_t)lmax) return cnt;
  flag_err(err, ERR_LIST);
  return (uint32_t)lmax;
}

// Classes (subsets of the split set D) that hold members: bit c set.
QR_HD uint64_t class_mask(uint64_t members, uint32_t D) {
  uint64_t cl = 0;
  for (uint64_t m = members; m; m &= m - 1) cl |= 1ull << (low_bit(m) & D);
  return cl;
}

// Split every class cl of the address (split set D, records from r0) on the
// tagged tokens X: class c gives c | y for every nonempty y within X (the
// tokens of y untagged and kept as entries, those of X \ y dropped) and
// keeps c (the tokens of X dropped).  The new split set D | X is written to
// every class slot touched and to the class-0 slot.
QR_HD void rec_class_split(uint16_t *r0, int rec, int k, int lmax, uint64_t cl, uint32_t D,
                           uint32_t X, uint32_t *err) {
  for (uint64_t m = cl; m; m &= m - 1) {
    const uint32_t c = low_bit(m);
    uint16_t *rc = r0 + (size_t)c * rec;
    const uint32_t cnt = rec_count(rc[0], lmax, err);
    const uint32_t busf = rc[1], toks = (busf >> 8) & 0xFFu, busm = busf & 0xFFu;
    for (uint32_t y = X; y; y = (y - 1) & X) {
      uint16_t *rn = r0 + (size_t)(c | y) * rec;
      uint32_t m2 = cnt;
      for (uint32_t j = 0; j < cnt; ++j) rn[2 + j] = rc[2 + j];
      for (int t = 0; t < k; ++t) {
        const uint32_t x = rc[2 + lmax + t];
        if (((y & toks) >> t) & 1u && x != REC_EMPTY) {  // kept: an ordinary entry now
          if (m2 < (uint32_t)lmax)
            rn[2 + m2++] = (uint16_t)x;
          else
            flag_err(err, ERR_LIST);
        }
        rn[2 + lmax + t] = ((X >> t) & 1u) ? (uint16_t)REC_EMPTY : (uint16_t)x;
      }
      rn[0] = (uint16_t)m2;
      rn[1] = (uint16_t)((busm & ~(X & ~y)) | ((toks & ~X) << 8));
      rn[2 + lmax + k] = (uint16_t)(D | X);
    }
    for (int t = 0; t < k; ++t)
      if ((X >> t) & 1u) rc[2 + lmax + t] = (uint16_t)REC_EMPTY;
    rc[0] = (uint16_t)cnt;
    rc[1] = (uint16_t)((busm & ~X) | ((toks & ~X) << 8));
    rc[2 + lmax + k] = (uint16_t)(D | X);
  }
  r0[2 + lmax + k] = (uint16_t)(D | X);
}

// Turn the members mc of class c into one ordinary list per component: bus
// word b gets the class's address entries plus the tagged tokens it carries
// (b & tokens) that are in the tree.  The class's own slot (bus word c) is
// rewritten last, since the others copy from it.  Marks the members' state
// words (st[wbase + b * nthr]) with W_SPLIT.
QR_HD void rec_split_class(uint16_t *r0, int rec, int k, int lmax, uint32_t c, uint64_t mc,
                           uint32_t *st, uint32_t wbase, uint32_t nthr, uint32_t *err) {
  uint16_t *rs = r0 + (size_t)c * rec;
  const uint32_t cnt = rec_count(rs[0], lmax, err);
  const uint32_t busf = rs[1], toks = (busf >> 8) & 0xFFu, busm = busf & 0xFFu;
  uint16_t tp[MAXK];
  for (int t = 0; t < k && t < MAXK; ++t) tp[t] = rs[2 + lmax + t];
  for (int pass = 0; pass < 2; ++pass) {
    for (uint64_t m = mc; m; m &= m - 1) {
      const uint32_t b = low_bit(m);
      if ((b == c) != (pass == 1)) continue;
      uint16_t *rb = r0 + (size_t)b * rec;
      if (b != c)
        for (uint32_t j = 0; j < cnt; ++j) rb[2 + j] = rs[2 + j];
      const uint32_t live = b & toks;
      uint32_t m2 = cnt;
      for (int t = 0; t < k && t < MAXK; ++t) {
        const uint32_t x = tp[t];
        if (!((live >> t) & 1u) || x == REC_EMPTY) continue;
        if (m2 < (uint32_t)lmax)
          rb[2 + m2++] = (uint16_t)x;
        else
          flag_err(err, ERR_LIST);
      }
      rb[0] = (uint16_t)m2;
      rb[1] = (uint16_t)(busm & (~toks | b));
      st[wbase + b * nthr] |= W_SPLIT;
    }
  }
}

}  // namespace qr
