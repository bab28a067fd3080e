// dco_layout.h -- sizes and per-pixel record layout that the aggregation
// kernels are built for (shared by host code and kernels; not part of the
// ABI).
#pragma once

#include <stdint.h>

// Largest arm length the kernels are built for.  The aggregation halo is
// 2 * kLMax columns/rows on each side of an output pixel.
constexpr int kLMax = 17;
// Threads of a streaming-aggregation workgroup = input columns of a strip.
constexpr int kStripThreads = 256;
// Output columns of one strip.
constexpr int kStripOut = kStripThreads - 4 * kLMax;

// Packed per-pixel records of one view for the aggregation kernels, written
// by k_geometry.  Both arrays hold 4-word entries (the fourth of b is unused:
// one 16-byte load per pixel is cheaper than a 12-byte one), Wp per row; column x
// sits at x + apron, and the apron columns are zero.  With hw(p) = 4 (r + 1) | 4 l << 8
// (horizontal arms as byte offsets) and ring offsets rb(p) = the byte offsets
// of prefix rows y + dn and y - u - 1 in a ring (16 bits each):
//   b row r (H + kLMax + 1 rows; the last is zero), read at stream row r:
//     two stages: m, rb1, hw(x, r) | (N1/2 | sh << 10) << 16    of pixel (x, r - kLMax)
//                 for its stage-1 rounding floor((S1 + N1/2) / N1) = ((S1 + N1/2) m) >> sh
//     one stage:  RN(1/N1) 2^-20, rb1, hw(x, r) | N1 << 16
//     (hw of row r is 0 from row H on; the rest is 0 above row kLMax)
//   c row y (H + 1 rows; row H is zero), two stages only:
//     rb2, RN(1/N2) 2^-20, hw | N2 << 16, N2 2^20 (float)        of pixel (x, y)
struct AggRecords {
    uint32_t* b;
    uint32_t* c;
    int Wp, apron;
};
constexpr int kRecApronL = 2 * kLMax;        // left apron of the records
constexpr int kRecApronR = kStripThreads;    // right apron (covers a strip's overhang)

// How the records address the LDS of the kernel that reads them: the row
// counts of its two rings, the value stored per ring slot (ring 1 in bytes,
// ring 2 in bytes or in 8-byte words) and the bytes of one prefix-row entry
// (the scale of the arm offsets in hw).  Slot value x (rows - 1) and
// hw x (kLMax + 1) must fit 16 and 8 bits.
struct RecGeom {
    int ring1, ring2;
    uint32_t step1, step2, hw;
};
