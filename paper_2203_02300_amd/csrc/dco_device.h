// dco_device.h -- device-side bodies of every stage of the plain matcher.
//
// The one-call kernels (k_census.hip, k_aggregate.hip, k_wta.hip) and the
// batched work-list kernels (k_batch.hip) run exactly these functions, so a
// pair matched alone and the same pair matched in a batch give the same bits.
// Each function takes its LDS as an explicit struct.
#pragma once

#include "dco_internal.h"

namespace dco {

// ===========================================================================
// Census codes and cross-support arms (Sec. 4.1; C_census of Eq. 1)
// ===========================================================================

constexpr int kCenTW = 64, kCenTH = 16;                                  // pixel tile
constexpr int kCenRW = kCenTW + 2 * kLMax, kCenRH = kCenTH + 2 * kLMax;  // staged RGB region
constexpr int kCenHW = 4, kCenHH = 4;  // census half-window limits
constexpr int kCenGW = kCenTW + 2 * kCenHW, kCenGH = kCenTH + 2 * kCenHH;

struct CensusLds {
    uint32_t rgb[kCenRH][kCenRW];
    uint32_t grey[kCenGH][kCenGW];
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// DPP move of v (lanes without a source read 0): row shifts 0x111..0x118,
// row broadcasts 0x142 (lane 15 of each row to the next row) and 0x143
// (lane 31 to rows 2 and 3).
template <unsigned Ctrl, unsigned RowMask>
__device__ inline uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, false);
}

__device__ inline uint32_t grey_of(uint32_t c) {
    uint32_t r = c & 0xffu, g = (c >> 8) & 0xffu, b = (c >> 16) & 0xffu;
    return (77u * r + 150u * g + 29u * b + 128u) >> 8;
}

// Largest per-channel absolute difference below tau?  With the centre's
// channels biased as A_c = a_c + tau - 1, |a_c - b_c| < tau holds exactly when
// the unsigned A_c - b_c is below 2 tau - 1, so one test is three byte
// subtractions, a max3 and a compare.
struct Centre {
    uint32_t r, g, b, lim;
};
__device__ inline Centre centre_of(uint32_t a, int tau) {
    const uint32_t t = (uint32_t)tau - 1;
    return Centre{(a & 0xffu) + t, ((a >> 8) & 0xffu) + t, ((a >> 16) & 0xffu) + t,
                  2u * (uint32_t)tau - 1u};
}
__device__ inline bool close_rgb(const Centre& c, uint32_t b) {
    const uint32_t dr = c.r - (b & 0xffu), dg = c.g - ((b >> 8) & 0xffu),
                   db = c.b - ((b >> 16) & 0xffu);
    return max(max(dr, dg), db) < c.lim;
}

// Census code of tile pixel (tx, ty) from the grey levels in LDS: bit k is
// set when neighbour k (row-major over the window, centre skipped) is darker
// than the centre.  The fixed-size form unrolls, so its LDS reads pipeline.
// Grey levels are below 256, so n - c is negative exactly when n < c: each
// bit enters as the sign of n - c with one funnel shift (alignbit), from the
// last neighbour back to the first, the upper bits in one word and the lower
// in another.
template <int HW, int HH>
__device__ inline uint64_t census_code(const CensusLds& S, int tx, int ty) {
    constexpr int kBits = (2 * HW + 1) * (2 * HH + 1) - 1;
    static_assert(kBits <= 64, "one 64-bit code");
    const uint32_t c = S.grey[ty + kCenHH][tx + kCenHW];
    uint32_t hi = 0, lo = 0;
#pragma unroll
    for (int k = kBits - 1; k >= 0; --k) {
        constexpr int kCentre = HH * (2 * HW + 1) + HW;
        const int n = k < kCentre ? k : k + 1;  // window index, centre skipped
        const int dy = n / (2 * HW + 1) - HH, dx = n % (2 * HW + 1) - HW;
        const uint32_t d = S.grey[ty + kCenHH + dy][tx + kCenHW + dx] - c;
        if (k >= 32)
            hi = __builtin_amdgcn_alignbit(hi, d, 31);
        else
            lo = __builtin_amdgcn_alignbit(lo, d, 31);
    }
    return (uint64_t)hi << 32 | lo;
}

__device__ inline uint64_t census_code_any(const CensusLds& S, int tx, int ty, int hw, int hh) {
    const uint32_t c = S.grey[ty + kCenHH][tx + kCenHW];
    uint64_t code = 0;
    int bit = 0;
    for (int dy = -hh; dy <= hh; ++dy)
        for (int dx = -hw; dx <= hw; ++dx) {
            if (dy == 0 && dx == 0) continue;
            code |= (uint64_t)(S.grey[ty + kCenHH + dy][tx + kCenHW + dx] < c) << bit;
            ++bit;
        }
    return code;
}

// One 64 x 16 tile at (x0, y0), NT threads (256: four pixels per thread;
// 1024: one).  The tile plus a kLMax apron (edge-clamped) is staged in LDS as
// packed RGB words; grey levels of the tile plus the census apron go to a
// second array.
//   grey:   Y = (77 R + 150 G + 29 B + 128) >> 8
//   census: bit k = Y(q_k) < Y(p), neighbours row-major without the centre
//   arms:   steps j = 1.. while inside, j <= L1 and max channel |diff| < tau1
template <int NT = 256>
__device__ inline __attribute__((always_inline)) void census_tile(
    const uint8_t* __restrict__ rgb, int W, int H, int cw, int ch, int L1, int tau1,
    uint64_t* __restrict__ census, uint32_t* __restrict__ arms, uint32_t* __restrict__ rgb_packed,
    uint4* __restrict__ pix, int x0, int y0, CensusLds& S) {
    static_assert(NT % 64 == 0 && (kCenTW * kCenTH) % NT == 0, "whole rows per pass");
    const int t = threadIdx.x;
    {   // stage the region: every load issued before any is stored
        constexpr int kN = (kCenRW * kCenRH + NT - 1) / NT;
        uint32_t v[kN];
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int i = min(t + NT * k, kCenRW * kCenRH - 1);
            const int ry = i / kCenRW, rx = i - ry * kCenRW;
            const int gx = clampi(x0 - kLMax + rx, 0, W - 1);
            const int gy = clampi(y0 - kLMax + ry, 0, H - 1);
            const uint8_t* p = rgb + 3 * ((size_t)gy * W + gx);
            v[k] = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
        }
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int i = t + NT * k;
            if (i < kCenRW * kCenRH) {
                const int ry = i / kCenRW;
                S.rgb[ry][i - ry * kCenRW] = v[k];
            }
        }
    }
    __syncthreads();
    for (int i = t; i < kCenGW * kCenGH; i += NT) {
        int gy = i / kCenGW, gx = i - gy * kCenGW;
        S.grey[gy][gx] = grey_of(S.rgb[gy + kLMax - kCenHH][gx + kLMax - kCenHW]);
    }
    __syncthreads();

    const int hw = cw >> 1, hh = ch >> 1;
    const int tx = t & 63;
    for (int k = 0; k < kCenTH / (NT / 64); ++k) {
        const int ty = (t >> 6) + (NT / 64) * k;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H) continue;
        const uint64_t code = cw == 9 && ch == 7
                                  ? census_code<4, 3>(S, tx, ty)
                                  : census_code_any(S, tx, ty, hw, hh);
        if (census) census[(size_t)y * W + x] = code;

        const int rx = tx + kLMax, ry = ty + kLMax;
        const uint32_t cp = S.rgb[ry][rx];
        // each arm: the closeness of all kLMax steps as a bit mask (the reads
        // are independent, so they pipeline), then the run of ones from
        // step 1, capped by L1 and the border
        const Centre cc = centre_of(cp, tau1);
        uint32_t ml = 0, mr = 0, mu = 0, md = 0;
#pragma unroll
        for (int j = 1; j <= kLMax; ++j) {
            ml |= (uint32_t)close_rgb(cc, S.rgb[ry][rx - j]) << (j - 1);
            mr |= (uint32_t)close_rgb(cc, S.rgb[ry][rx + j]) << (j - 1);
            mu |= (uint32_t)close_rgb(cc, S.rgb[ry - j][rx]) << (j - 1);
            md |= (uint32_t)close_rgb(cc, S.rgb[ry + j][rx]) << (j - 1);
        }
        const int al = min(min(L1, x), __builtin_ctz(~ml));
        const int ar = min(min(L1, W - 1 - x), __builtin_ctz(~mr));
        const int au = min(min(L1, y), __builtin_ctz(~mu));
        const int ad = min(min(L1, H - 1 - y), __builtin_ctz(~md));
        arms[(size_t)y * W + x] =
            (uint32_t)al | ((uint32_t)ar << 8) | ((uint32_t)au << 16) | ((uint32_t)ad << 24);
        if (rgb_packed) rgb_packed[(size_t)y * W + x] = cp;
        // everything the fused raw cost needs of one pixel in one 16-byte
        // load: census code, packed RGB, and 8 L_min (the byte offset of the
        // pixel's (alpha, beta) pair)
        if (pix)
            pix[(size_t)y * W + x] = make_uint4((uint32_t)code, (uint32_t)(code >> 32), cp,
                                                (uint32_t)(8 * min(min(al, ar), min(au, ad))));
    }
}

// ===========================================================================
// Region counts and packed aggregation records of one pixel
// ===========================================================================
//   N1 = sum over y' in [y-u, y+dn] of (l(x,y') + r(x,y') + 1)
//   N2 = sum over x' in [x-l, x+r] of (u(x',y) + dn(x',y) + 1)
// Stage-1 rounding uses sh = 31 + ceil(log2 N1) and m = ceil(2^sh / N1) <
// 2^32, so floor(n / N1) = (n * m) >> sh for every 0 <= n < 2^31 (N1 <= 2^11).
// A final division by N uses N' = N * 2^20 and y' = RN(1/N) * 2^-20 (both
// exact scalings), so that it also removes the Q20 scale (div_q20 below).
//
// The streaming kernel keeps row r of a column-prefix ring in slot r mod R,
// so the byte offsets of the two prefix rows of a vertical range are fixed
// per pixel and are stored here (16 bits each).

constexpr int kAggK = kStripThreads / 64;             // rows per chunk = wavefronts (4)
constexpr int kSeg = kStripThreads / 64;              // 64-column segments of a strip row
constexpr int kRing1 = 2 * kLMax + 1 + kAggK;         // stage-1 prefix rows per column
constexpr int kRing2 = 2 * kLMax + 2 + kAggK;         // stage 2 is read one chunk later
constexpr int kRingCols = kStripThreads - 2 * kLMax;  // columns with a ring: 222
constexpr int kRingStride = 224;                      // a multiple of the 32 LDS banks
constexpr uint32_t kSlotBytes = kRingStride * 4;
constexpr int kPStride = 280;                         // prefix row: P(-1) at 0, P(i) at i + 1
constexpr uint32_t kOOB = 0x7fffffffu;                // buffer offset that reads as 0
static_assert(kRing2 * kSlotBytes < 65536, "ring offsets are stored in 16 bits");
static_assert(kStripThreads == 256 && kAggK == 4, "one row per wavefront per chunk");

__device__ inline uint32_t ring_slot(int row, int ring) {
    int s = row % ring;
    if (s < 0) s += ring;
    return (uint32_t)s;
}
__device__ inline uint32_t ring_slot_bytes(int row, int ring) {
    return ring_slot(row, ring) * kSlotBytes;
}

// Records for the single-slice kernels (k_agg_stream, k_agg_pair<1>, the
// batched path).
constexpr RecGeom kRecPlain{kRing1, kRing2, kSlotBytes, kSlotBytes, 4};

// Records of pixel (x, y) with arms word a and region counts n1, n2 (layout:
// AggRecords).  The b row of the pixel's own row gets its horizontal arms
// (low half of word 2); the b row kLMax rows below gets its stage-1 data.
// ring1 and ring2 are the row counts of the two rings of the kernel that
// reads the records.
__device__ inline void write_records(const AggRecords& rec, int x, int y, int iters, uint32_t a,
                                     uint32_t n1, uint32_t n2, const RecGeom& g) {
    const uint32_t l = a & 0xff, r = (a >> 8) & 0xff, u = (a >> 16) & 0xff, dn = a >> 24;
    const uint32_t lr = g.hw * (r + 1) | (g.hw * l) << 8;
    const uint32_t hi = (uint32_t)y + dn, lo = (uint32_t)y - u - 1;
    const size_t col = (size_t)x + rec.apron;
    uint32_t* bo = rec.b + 4 * ((size_t)y * rec.Wp + col);
    reinterpret_cast<uint16_t*>(bo + 2)[0] = (uint16_t)lr;
    uint32_t* bv = rec.b + 4 * ((size_t)(y + kLMax) * rec.Wp + col);
    bv[1] = ring_slot((int)hi, g.ring1) * g.step1 | ring_slot((int)lo, g.ring1) * g.step1 << 16;
    if (iters == 2) {
        const uint32_t lg = n1 <= 1 ? 0u : 32u - (uint32_t)__clz((int)(n1 - 1));
        const uint32_t sh = 31u + lg;
        // m = ceil(2^sh / N1) from the correctly rounded double quotient:
        // the quotient is below 2^32, so its rounding error is at most 2^-22,
        // while a quotient that is not an integer is at least 1 / N1 > 2^-11
        // away from one, so the ceiling is exact
        bv[0] = (uint32_t)__builtin_ceil(__builtin_ldexp(1.0, (int)sh) / (double)n1);
        reinterpret_cast<uint16_t*>(bv + 2)[1] = (uint16_t)((n1 >> 1) | sh << 10);
        uint32_t* c = rec.c + 4 * ((size_t)y * rec.Wp + col);
        c[0] = ring_slot((int)hi, g.ring2) * g.step2 | ring_slot((int)lo, g.ring2) * g.step2 << 16;
        c[1] = __float_as_uint((1.0f / (float)n2) * 0x1p-20f);
        c[2] = lr | n2 << 16;
        c[3] = __float_as_uint((float)n2 * 0x1p20f);
    } else {
        bv[0] = __float_as_uint((1.0f / (float)n1) * 0x1p-20f);
        reinterpret_cast<uint16_t*>(bv + 2)[1] = (uint16_t)n1;
    }
}

// Region counts and records of a 64 x 16 tile at (x0, y0), 256 threads.  The
// arms of the tile plus a kLMax apron go to LDS as h = l + r + 1 and
// v = u + dn + 1; prefix sums of h down each tile column and of v along each
// tile row then give every N1 and N2 with two reads.  Apron cells outside the
// image hold 0 and never fall inside a region (arms stop at the border).
constexpr int kGeoTW = 64, kGeoTH = 16;
constexpr int kGeoRW = kGeoTW + 2 * kLMax, kGeoRH = kGeoTH + 2 * kLMax;

struct GeomLds {
    uint32_t hv[kGeoRH][kGeoRW];       // h | v << 16
    uint32_t cp[kGeoRH + 1][kGeoTW];   // column prefixes of h (row 0 = 0)
    uint32_t rp[kGeoTH][kGeoRW + 1];   // row prefixes of v (column 0 = 0)
};

// NT = 256 threads sum the prefixes with one thread per column or row;
// NT = 1024 threads use DPP scans (16 lanes per column, one wavefront per
// row) and take one pixel each.
template <int NT = 256>
__device__ inline __attribute__((always_inline)) void geometry_tile(
    const uint32_t* __restrict__ arms, int W, int H, int iters, const AggRecords& rec, int x0,
    int y0, GeomLds& S, const RecGeom& g = kRecPlain) {
    static_assert(NT == 256 || NT == 1024, "256 or 1024 threads");
    const int t = threadIdx.x;
    {   // stage the arms: every load issued before any is used (clamped addresses)
        constexpr int kN = (kGeoRW * kGeoRH + NT - 1) / NT;
        uint32_t v[kN];
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int i = min(t + NT * k, kGeoRW * kGeoRH - 1);
            const int ry = i / kGeoRW, rx = i - ry * kGeoRW;
            const int x = clampi(x0 - kLMax + rx, 0, W - 1), y = clampi(y0 - kLMax + ry, 0, H - 1);
            v[k] = arms[(size_t)y * W + x];
        }
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int i = t + NT * k;
            if (i < kGeoRW * kGeoRH) {
                const int ry = i / kGeoRW, rx = i - ry * kGeoRW;
                const int x = x0 - kLMax + rx, y = y0 - kLMax + ry;
                const uint32_t a = v[k];
                S.hv[ry][rx] = x >= 0 && x < W && y >= 0 && y < H
                                   ? ((a & 0xff) + ((a >> 8) & 0xff) + 1) |
                                         ((a >> 16 & 0xff) + (a >> 24) + 1) << 16
                                   : 0u;
            }
        }
    }
    __syncthreads();
    if constexpr (NT == 256) {
        if (t < kGeoTW) {  // column prefixes of h
            uint32_t acc = 0;
            S.cp[0][t] = 0;
#pragma unroll 10
            for (int ry = 0; ry < kGeoRH; ++ry) {
                acc += S.hv[ry][t + kLMax] & 0xffff;
                S.cp[ry + 1][t] = acc;
            }
        } else if (t < kGeoTW + kGeoTH) {  // row prefixes of v
            const int ty = t - kGeoTW;
            uint32_t acc = 0;
            S.rp[ty][0] = 0;
#pragma unroll 14
            for (int rx = 0; rx < kGeoRW; ++rx) {
                acc += S.hv[ty + kLMax][rx] >> 16;
                S.rp[ty][rx + 1] = acc;
            }
        }
    } else {
        {   // column prefixes of h: column c = t / 16, rows 4 s .. 4 s + 3 with
            // s = t % 16 (16 lanes = one DPP row per column)
            const int c = t >> 4, sg = t & 15;
            uint32_t a[4], tot = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ry = 4 * sg + i;
                tot += ry < kGeoRH ? S.hv[ry][c + kLMax] & 0xffff : 0u;
                a[i] = tot;
            }
            uint32_t inc = tot;
            inc += dpp<0x111, 0xf>(inc);
            inc += dpp<0x112, 0xf>(inc);
            inc += dpp<0x114, 0xf>(inc);
            inc += dpp<0x118, 0xf>(inc);
            const uint32_t before = inc - tot;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ry = 4 * sg + i;
                if (ry < kGeoRH) S.cp[ry + 1][c] = before + a[i];
            }
            if (sg == 0) S.cp[0][c] = 0;
        }
        {   // row prefixes of v: wavefront w takes row w, lane l columns 2 l, 2 l + 1
            const int ty = t >> 6, l = t & 63;
            const uint32_t v0 = 2 * l < kGeoRW ? S.hv[ty + kLMax][2 * l] >> 16 : 0u;
            const uint32_t v1 = 2 * l + 1 < kGeoRW ? S.hv[ty + kLMax][2 * l + 1] >> 16 : 0u;
            const uint32_t tot = v0 + v1;
            uint32_t inc = tot;
            inc += dpp<0x111, 0xf>(inc);
            inc += dpp<0x112, 0xf>(inc);
            inc += dpp<0x114, 0xf>(inc);
            inc += dpp<0x118, 0xf>(inc);
            inc += dpp<0x142, 0xa>(inc);
            inc += dpp<0x143, 0xc>(inc);
            const uint32_t before = inc - tot;
            if (2 * l < kGeoRW) S.rp[ty][2 * l + 1] = before + v0;
            if (2 * l + 1 < kGeoRW) S.rp[ty][2 * l + 2] = before + tot;
            if (l == 0) S.rp[ty][0] = 0;
        }
    }
    __syncthreads();
    const int tx = t & 63;
    const int x = x0 + tx;
    for (int k = 0; k < kGeoTH / (NT / 64); ++k) {
        const int ty = (t >> 6) + (NT / 64) * k;
        const int y = y0 + ty;
        if (x >= W || y >= H) continue;
        // arms from census_tile never exceed kLMax; the clamp only keeps an
        // arbitrary caller-supplied arms map from indexing outside the tile
        const uint32_t a0 = arms[(size_t)y * W + x];
        const int l = min((int)(a0 & 0xff), kLMax), r = min((int)((a0 >> 8) & 0xff), kLMax);
        const int u = min((int)((a0 >> 16) & 0xff), kLMax), dn = min((int)(a0 >> 24), kLMax);
        const uint32_t a = (uint32_t)l | (uint32_t)r << 8 | (uint32_t)u << 16 | (uint32_t)dn << 24;
        const uint32_t n1 = S.cp[ty + kLMax + dn + 1][tx] - S.cp[ty + kLMax - u][tx];
        const uint32_t n2 = S.rp[ty][tx + kLMax + r + 1] - S.rp[ty][tx + kLMax - l];
        write_records(rec, x, y, iters, a, n1, n2, g);
    }
}

// ===========================================================================
// Streaming two-stage aggregation (Eq. 2 twice), one slice x one column strip
// ===========================================================================
//
// A strip is 256 consecutive columns: 2 kLMax apron columns on each side and
// kStripOut output columns in the middle.  The workgroup streams down the
// rows in chunks of kAggK = 4 rows, in three steps per chunk:
//   1 (wavefront w, row yc + w, all 256 columns as 4 segments of 64):
//       raw cost q (fused: Eq. 1 from the images; staged: read), inclusive
//       row prefix P1 by a wavefront scan per segment plus segment carries
//   2 (thread t owns column t, rows yc .. yc + 3 in order):
//       H1: E1 = P1(t + r) - P1(t - l - 1); push the column prefix of E1
//       V1: S1 of row y - kLMax from two prefix rows of ring 1
//           a1 = floor((S1 + N1/2) / N1) (multiply-shift), push into ring 2
//   3 (wavefront w, output row y - 2 kLMax - 1 of row yc + w, 4 segments):
//       V2: E2 from two prefix rows of ring 2; row prefix P2 as in step 1
//       H2: S2 = P2(t + r) - P2(t - l - 1); out = RN(S2 / N2) * 2^-20
// Two barriers per chunk: after step 1 (P1 rows) and after step 2 (ring 2,
// and the end of step 2's reads of P1).  Row prefixes of steps 1 and 3 share
// one LDS row per wavefront: only the wavefront that owns a row writes it.
// Ring 1 holds kAggK - 1 rows more than a vertical range spans so that a
// chunk's four pushes can precede its four range reads; ring 2 is read in
// step 3, after all four pushes of step 2, so it holds kAggK rows more.
//
// Every sum is an integer and differences of prefix sums are taken mod 2^32
// (every true range sum is below 2^31), so the result does not depend on the
// summation order, and a band of output rows [y0, y1) can start from zero
// prefixes 2 kLMax + 1 rows above y0: the rows before the start then shift
// every prefix by the same constant.
//
// Per-pixel data comes from padded records (zero apron, zero row H) through
// buffer loads with a per-lane column offset and a uniform row offset, so the
// chunk body has no bounds branches.

// Every member starts below 64 KB, so LDS addresses fold into the 16-bit
// instruction offsets.  Reads of a prefix row reach up to kLMax words before
// it (apron lanes, results unused): `guard` and the tables keep them inside
// the allocation.
template <int ITERS, bool kFused>
struct AggLds {
    float tabA[kFused ? 768 : 1];
    float tabC[kFused ? 68 : 1];
    float2 ab[kFused ? kLMax + 1 : 1];
    uint32_t guard[32];
    uint32_t prow[kAggK][kPStride];
    uint32_t ring1[kRing1 * kRingStride];
    uint32_t ring2[ITERS == 2 ? kRing2 * kRingStride : 1];
};

typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ inline rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ inline uint32_t ld32(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
__device__ inline uint4 ld128(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
// Stores of the aggregated volume are non-temporal (the volume is streamed to
// HBM and read once by WTA), so they do not evict reused inputs from L2.
__device__ inline void st32(float v, rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 2);
}

// Inclusive prefix sums of the kSeg segments across the wavefront: DPP row
// shifts 1, 2, 4, 8 and the gfx9 row broadcasts 15 and 31, step-major so the
// segments interleave; then each segment adds the totals of the ones before.
__device__ inline void wave_scan_segments(uint32_t (&v)[kSeg]) {
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x111, 0xf>(v[j]);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x112, 0xf>(v[j]);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x114, 0xf>(v[j]);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x118, 0xf>(v[j]);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x142, 0xa>(v[j]);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) v[j] += dpp<0x143, 0xc>(v[j]);
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const uint32_t tot = __builtin_amdgcn_readlane(v[j], 63);
        v[j] += carry;
        carry += tot;
    }
}

// Wavefront index inside the workgroup, known to the compiler as uniform.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

__device__ inline uint32_t lds_ld(const uint32_t* base, uint32_t byte_off) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ inline void lds_st(uint32_t* base, uint32_t byte_off, uint32_t v) {
    *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// One Q20 term of Eq. 1, rint(a t) rounded once from the exact product of
// the float factors (a carries the 2^20 scale), for 0 <= a t < 2^22: the
// fused a t + 2^23 rounds to 2^23 + rint(a t), whose float bits are
// 0x4B000000 + rint(a t).
__device__ inline uint32_t q20_term(float a, float t) {
    return __builtin_bit_cast(uint32_t, __builtin_fmaf(a, t, 0x1p23f)) - 0x4B000000u;
}

// RN((float)s / N) * 2^-20 given N' = N * 2^20 and y' = RN(1/N) * 2^-20.
// With y = RN(1/N): q0 = RN(s * y) is within two ulps of s/N, r = s - q0 * N
// is then exact, and s/N is never a float midpoint for integer N, so
// RN(q0 + r * y) = RN(s / N).  Scaling y and q0 by 2^-20 and N by 2^20 is
// exact and commutes with the roundings (no result is subnormal).
__device__ inline float div_q20(uint32_t s, float n_scaled, float rcp_scaled) {
    const float a = (float)s;
    const float q0 = a * rcp_scaled;
    const float r = __builtin_fmaf(-q0, n_scaled, a);
    return __builtin_fmaf(r, rcp_scaled, q0);
}

struct AggArgs {
    const float* cost;         // staged: D x H x W raw costs
    const uint4* pixL;         // fused: packed pixels of both views (H x W):
    const uint4* pixR;         //   census lo, census hi, RGB, 8 L_min
    const float* tabA;         // fused: Eq. 1 tables
    const float* tabC;
    const float* alpha;
    const float* beta;
    AggRecords rec;            // padded per-pixel records of the reference view
    float* out;                // D x H x W
    // two-slice kernel: store `out` in the paired layout (see paired_at)
    bool paired;
    int W, H, D, nstrips, ref, L1;
};

// Paired layout of a D-slice cost volume: for each pixel and pair of slices
// (2g, 2g + 1), slice 2g holds the bits of the smaller cost (the first on a
// tie; costs are >= 0, so bit 31 is free) with bit 31 set when that is slice
// 2g + 1's, and slice 2g + 1 holds the other cost.  A last slice without a
// partner (odd D) holds its cost as it is.  Winner-take-all then reads only
// the even slices.  paired_at returns the cost of slice s at pixel i.
__device__ inline float paired_at(const float* __restrict__ vol, int P, int D, int s, int i) {
    const int e = s & ~1;
    const uint32_t w = __builtin_bit_cast(uint32_t, vol[(size_t)e * P + i]);
    if (e + 1 >= D || (s & 1) == (int)(w >> 31))
        return __builtin_bit_cast(float, w & 0x7fffffffu);
    return vol[(size_t)(e + 1) * P + i];
}

// Loads of one chunk.  Step 1 and step 3 loads are for this lane's four
// segment columns of its wavefront's row; step 2 loads are for the owned
// column and the chunk's four rows.
template <bool kFused>
struct ChunkIn {
    uint4 ref[kSeg];            // fused: reference pixel; staged: .x = raw cost bits
    uint4 par[kSeg];            // fused: partner pixel
    uint4 b2[kAggK];            // step 2: records b of rows yc + k
    uint4 c3[kSeg];             // step 3: records c of the output row
};

// Per-lane constants of a strip.
struct AggLane {
    uint32_t img[kSeg];   // byte offset of each segment column in an H x W row (packed
                          // pixels: x16; cost slice: x4), or kOOB
    uint32_t par[kSeg];   // fused: the partner column's byte offset, or kOOB
    uint32_t inval[kSeg]; // fused: raw cost when the partner is outside (2^20; 0 off-image)
    uint32_t recw;        // record column index x4 of segment 0 of this lane
    uint32_t reco;        // record column index x4 of the owned column
    uint32_t cb1, cb2;    // ring byte offsets of the owned column
    uint32_t cbs[kSeg];   // ring-2 byte offset of each segment column (column
                          // kRingCols + 1, never written, for columns without a ring)
    uint32_t vout[kSeg];  // output byte offset of each segment column, or kOOB
    uint32_t vout_o;      // output byte offset of the owned column, or kOOB (one stage)
    bool pok[kSeg];       // fused: partner inside the image
};

struct AggRes {
    rsrc_t rB, rC, rq, rIr, rIp, rOut;
    uint32_t slice_bytes;  // two-slice kernel: distance between its output slices
    uint32_t in_slice_bytes;  // staged two-slice kernel: distance between its input
                              // slices (0 when only one slice is left: it is read twice)
    int nout;              // two-slice kernel: slices that exist (the others are not stored)
    bool paired;           // two-slice kernel: paired layout (AggArgs::paired)
};

template <int ITERS, bool kFused>
__device__ inline void load_chunk(const AggArgs& A, int yc, const AggLane& ln, const AggRes& R,
                                  ChunkIn<kFused>& in) {
    const int H = A.H;
    const uint32_t Wp = (uint32_t)A.rec.Wp, W = (uint32_t)A.W;
    const int w = wave_id();
    {   // step 1: row yc + w
        const int y = yc + w;
        const uint32_t yq = (uint32_t)min(y, H - 1);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            if (kFused) {
                in.ref[j] = ld128(R.rIr, ln.img[j], yq * W * 16);
                in.par[j] = ld128(R.rIp, ln.par[j], yq * W * 16);
            } else {
                in.ref[j].x = ld32(R.rq, ln.img[j], yq * W * 4);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {  // step 2: b row yc + k (rows past the last read zeros)
        const int y = yc + k;
        const uint32_t rb = (uint32_t)min(y, H + kLMax);
        in.b2[k] = ld128(R.rB, ln.reco * 4, rb * Wp * 16);
    }
    if (ITERS == 2) {  // step 3: output row yc + w - 2 kLMax - 1
        const int y2 = yc + w - 2 * kLMax - 1;
        const uint32_t rc = (uint32_t)(y2 >= 0 && y2 < H ? y2 : H);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) in.c3[j] = ld128(R.rC, ln.recw * 4 + 1024 * j, rc * Wp * 16);
    }
}

template <int ITERS, bool kFused>
__device__ inline void process_chunk(const AggArgs& A, int yc, int y0, int y1, const AggLane& ln,
                                     const AggRes& R, const ChunkIn<kFused>& in,
                                     uint32_t& cp1, uint32_t& cp2, uint32_t& s1off,
                                     uint32_t& s2off, AggLds<ITERS, kFused>& S) {
    const int t = threadIdx.x, w = wave_id(), lane = t & 63;
    const int H = A.H, W = A.W;
    uint32_t* prow_w = S.prow[w];
    // ---- step 1: raw costs and row prefixes of row yc + w ----
    {
        const int y = yc + w;
        uint32_t v[kSeg];
        if (y < H) {  // uniform: rows below the image contribute nothing
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                if (kFused) {
                    const uint32_t s = __builtin_amdgcn_sad_u8(in.ref[j].z, in.par[j].z, 0u);
                    const uint64_t x = ((uint64_t)in.ref[j].y << 32 | in.ref[j].x) ^
                                       ((uint64_t)in.par[j].y << 32 | in.par[j].x);
                    const uint32_t h = (uint32_t)__popcll(x);
                    const float2 ab = *reinterpret_cast<const float2*>(
                        reinterpret_cast<const char*>(S.ab) + in.ref[j].w);
                    uint32_t q = q20_term(ab.x, S.tabA[s]) + q20_term(ab.y, S.tabC[h]);
                    // keep the lookups unconditional (interleaved across
                    // segments); the select is then one lane-mask cndmask
                    asm volatile("" : "+v"(q));
                    v[j] = ln.pok[j] ? q : ln.inval[j];
                } else {
                    v[j] = (uint32_t)(__builtin_bit_cast(float, in.ref[j].x) * 1048576.0f);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < kSeg; ++j) v[j] = 0u;
        }
        wave_scan_segments(v);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) prow_w[64 * j + lane + 1] = v[j];
    }
    __syncthreads();
    // ---- step 2: column prefixes, stage-1 means of rows yc + k - kLMax ----
    // Ring 1 keeps kAggK - 1 rows more than a range needs, so the chunk's
    // four pushes can all go before its four range reads.
    uint32_t e1[kAggK], s1[kAggK];
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint32_t a = in.b2[k].z;
        const uint32_t pb = (uint32_t)(k * kPStride + t) * 4;
        e1[k] = lds_ld(S.prow[0], pb + (a & 0xff)) - lds_ld(S.prow[0], pb - ((a >> 8) & 0xff));
    }
    uint32_t off = s1off;
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        cp1 += e1[k];
        lds_st(S.ring1, ln.cb1 + off, cp1);
        off = off + kSlotBytes == kRing1 * kSlotBytes ? 0u : off + kSlotBytes;
    }
    s1off = off;
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint32_t o = in.b2[k].y;
        s1[k] = lds_ld(S.ring1, ln.cb1 + (o & 0xffff)) - lds_ld(S.ring1, ln.cb1 + (o >> 16));
    }
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint4 b = in.b2[k];
        if (ITERS == 2) {
            const uint64_t n = (uint64_t)(s1[k] + ((b.z >> 16) & 1023)) * b.x;
            cp2 += (uint32_t)(n >> (b.z >> 26));
            lds_st(S.ring2, ln.cb2 + s2off, cp2);
            s2off = s2off + kSlotBytes == kRing2 * kSlotBytes ? 0u : s2off + kSlotBytes;
        } else {
            const int yv = yc + k - kLMax;
            const float a1 = div_q20(s1[k], (float)(b.z >> 16) * 0x1p20f,
                                     __builtin_bit_cast(float, b.x));
            if (yv >= y0 && yv < y1) st32(a1, R.rOut, ln.vout_o, (uint32_t)(yv * W) * 4);
        }
    }
    __syncthreads();
    if (ITERS == 2) {
        // ---- step 3: stage-2 means of output row yc + w - 2 kLMax - 1 ----
        const int y2 = yc + w - 2 * kLMax - 1;
        uint32_t v[kSeg];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t o = in.c3[j].x;
            v[j] = lds_ld(S.ring2, ln.cbs[j] + (o & 0xffff)) -
                   lds_ld(S.ring2, ln.cbs[j] + (o >> 16));
        }
        wave_scan_segments(v);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) prow_w[64 * j + lane + 1] = v[j];
        // the row was written by this wavefront only: LDS keeps its order
        float out[kSeg];
        const uint32_t pbw = (uint32_t)(w * kPStride + lane) * 4;
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t lr = in.c3[j].z;
            const uint32_t s2 = lds_ld(S.prow[0], pbw + 256 * j + (lr & 0xff)) -
                                lds_ld(S.prow[0], pbw + 256 * j - ((lr >> 8) & 0xff));
            out[j] = div_q20(s2, (float)(in.c3[j].z >> 16) * 0x1p20f,
                             __builtin_bit_cast(float, in.c3[j].y));
        }
        if (y2 >= y0 && y2 < y1) {
#pragma unroll
            for (int j = 0; j < kSeg; ++j) st32(out[j], R.rOut, ln.vout[j], (uint32_t)(y2 * W) * 4);
        }
    }
}

// Output rows [y0, y1) of slice d and column strip `strip` (256 threads).
template <int ITERS, bool kFused>
__device__ inline void agg_stream(const AggArgs& A, int d, int strip, int y0, int y1,
                                  AggLds<ITERS, kFused>& S) {
    const int W = A.W, H = A.H;
    const int t = threadIdx.x, lane = t & 63;
    const int x0 = strip * kStripOut;
    const size_t slice = (size_t)W * H;

    if (kFused) {
        for (int i = t; i < 766; i += kStripThreads) S.tabA[i] = A.tabA[i];
        if (t < 65) S.tabC[t] = A.tabC[t];
        if (t <= kLMax) {
            const int L = min(t, A.L1);
            S.ab[t] = make_float2(A.alpha[L], A.beta[L]);
        }
    }
    if (t < kAggK) S.prow[t][0] = 0;  // P(-1) of every prefix row
    // zero column prefixes: rows before the start contribute nothing
    for (int i = t; i < kRing1 * kRingStride; i += kStripThreads) S.ring1[i] = 0;
    if (ITERS == 2)
        for (int i = t; i < kRing2 * kRingStride; i += kStripThreads) S.ring2[i] = 0;

    AggLane ln;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const int i = 64 * j + lane;            // strip column of segment j
        const int c = x0 - 2 * kLMax + i;       // image column
        const bool in_img = c >= 0 && c < W;
        const int cp = A.ref == 0 ? c - d : c + d;
        const bool pok = in_img && cp >= 0 && cp < W;
        ln.img[j] = in_img ? (uint32_t)c * (kFused ? 16 : 4) : kOOB;
        ln.par[j] = pok ? (uint32_t)cp * 16 : kOOB;
        ln.pok[j] = pok;
        ln.inval[j] = in_img ? (1u << 20) : 0u;
        const bool rok = i >= kLMax && i < kLMax + kRingCols;
        ln.cbs[j] = (uint32_t)(rok ? i - kLMax : kRingCols + 1) * 4;
        ln.vout[j] = i >= 2 * kLMax && i < 2 * kLMax + kStripOut && c < W ? (uint32_t)c * 4 : kOOB;
    }
    {
        const int c = x0 - 2 * kLMax + t;
        const int jj = t - kLMax;
        const bool ring = jj >= 0 && jj < kRingCols;
        // owners without a ring column share one scratch column; column
        // kRingCols + 1 stays zero
        ln.cb1 = (uint32_t)(ring ? jj : kRingCols) * 4;
        ln.cb2 = ln.cb1;
        ln.reco = (uint32_t)(c + A.rec.apron) * 4;
        ln.recw = (uint32_t)(x0 - 2 * kLMax + lane + A.rec.apron) * 4;
        ln.vout_o = t >= 2 * kLMax && t < 2 * kLMax + kStripOut && c < W ? (uint32_t)c * 4 : kOOB;
    }
    const uint32_t recN = (uint32_t)(A.rec.Wp * (H + 1));
    const uint32_t P4 = (uint32_t)(slice * 4);
    const uint4* Iref = A.ref == 0 ? A.pixL : A.pixR;
    const uint4* Ipar = A.ref == 0 ? A.pixR : A.pixL;
    AggRes R;
    R.rB = make_rsrc(A.rec.b, (uint32_t)(A.rec.Wp * (H + kLMax + 1)) * 16);
    R.rC = make_rsrc(ITERS == 2 ? (const void*)A.rec.c : (const void*)A.rec.b,
                     ITERS == 2 ? recN * 16 : 0u);
    R.rq = make_rsrc(kFused ? (const void*)A.rec.b : (const void*)(A.cost + (size_t)d * slice),
                     kFused ? 0u : P4);
    R.rIr = make_rsrc(kFused ? (const void*)Iref : (const void*)A.rec.b, kFused ? 4 * P4 : 0u);
    R.rIp = make_rsrc(kFused ? (const void*)Ipar : (const void*)A.rec.b, kFused ? 4 * P4 : 0u);
    R.rOut = make_rsrc(A.out + (size_t)d * slice, P4);
    __syncthreads();

    // warm-up rows so that the first output row sees complete ranges
    const int warm = ITERS == 2 ? 2 * kLMax + 1 : kLMax;
    const int ys = max(0, y0 - warm);
    const int yend = y1 + warm;
    uint32_t cp1 = 0, cp2 = 0;
    uint32_t s1off = ring_slot_bytes(ys, kRing1);
    uint32_t s2off = ring_slot_bytes(ys - kLMax, kRing2);
    ChunkIn<kFused> ca, cb;
    load_chunk<ITERS, kFused>(A, ys, ln, R, ca);
    for (int yc = ys; yc < yend; yc += 2 * kAggK) {
        // the next chunk's loads are in flight while this chunk is processed
        load_chunk<ITERS, kFused>(A, yc + kAggK, ln, R, cb);
        process_chunk<ITERS, kFused>(A, yc, y0, y1, ln, R, ca, cp1, cp2, s1off, s2off, S);
        if (yc + kAggK >= yend) break;
        load_chunk<ITERS, kFused>(A, yc + 2 * kAggK, ln, R, ca);
        process_chunk<ITERS, kFused>(A, yc + kAggK, y0, y1, ln, R, cb, cp1, cp2, s1off, s2off,
                                     S);
    }
}

// ===========================================================================
// Two-slice streaming aggregation with specialised wavefronts (one-call path)
// ===========================================================================
//
// One workgroup of 512 threads streams two adjacent disparity slices of one
// column strip down the rows, in chunks of kAggK rows as above, with each
// step done by a fixed set of wavefronts and the steps of three consecutive
// chunks in flight:
//   row wavefronts 0-3, phase p: step 3 of chunk p - 2 (its output row,
//       both slices) and step 1 of chunk p (its row, both slices);
//   column wavefronts 4-7 (thread 256 + t owns column t), phase p: step 2 of
//       chunk p - 1 (both slices).
// One barrier ends a phase.  Each step's reference pixels and records are
// loaded once for both slices, and every LDS word holds the two slices'
// values of one column (one 64-bit access serves both).
//  * Prefix rows are double-buffered by chunk parity: step 1 of chunk p
//    writes buffer p & 1 while step 2 of chunk p - 1 reads the other one.
//    Step 3 uses its own wavefront's row of buffer p & 1 as scratch before
//    step 1 of the same wavefront overwrites it.
//  * Ring 1 is private to the column thread, which pushes a row and reads
//    that row's range before the next push, so 2 kLMax + 2 rows suffice.
//  * Ring 2 is pushed by step 2 of chunk p - 1 while step 3 of chunk p - 2
//    reads it: it keeps 2 kLMax + 2 + 2 kAggK rows so that no push of the
//    phase lands on a row still being read.
constexpr int kWsThreads = 2 * kStripThreads;
constexpr int kWsSlices = 2;
static_assert(kWsSlices == 2 && kSeg == 4, "the step-1 register pin lists 2 x 4 values");
constexpr int kWsRing1 = 2 * kLMax + 2;
constexpr int kWsRing2 = 2 * kLMax + 2 + 2 * kAggK;
constexpr uint32_t kWsSlotBytes = kRingStride * 8;  // one ring row of both slices
// Prefix rows hold P(c) at index c + kWsP0 and P(-1) = 0 at kWsP0 - 1, so
// that lane l's four columns 4 l .. 4 l + 3 form two aligned 16-byte words.
constexpr int kWsP0 = 4;
constexpr int kWsPStride = 260;  // P(-1) .. P(255)
static_assert(kWsPStride % 2 == 0 && kWsP0 + 256 <= kWsPStride, "prefix row layout");
// Records for this kernel: ring 1 offsets in bytes, ring 2 offsets in 8-byte
// words (its byte offsets would not fit 16 bits), arm offsets in 8-byte words.
constexpr RecGeom kRecWs{kWsRing1, kWsRing2, kWsSlotBytes, kRingStride, 8};
static_assert((kWsRing1 - 1) * kWsSlotBytes < 65536 && (kWsRing2 - 1) * kRingStride < 65536,
              "ring offsets are stored in 16 bits");

struct AggLdsWs {
    float tabA[768];
    float tabC[68];
    float2 ab[kLMax + 1];
    uint32_t guard[32];
    alignas(16) uint2 prow[2][kAggK][kWsPStride];  // [buffer][row][index]: both slices
    uint2 ring1[kWsRing1 * kRingStride];            // [slot][column]: both slices
    uint2 ring2[kWsRing2 * kRingStride];
};
static_assert(sizeof(AggLdsWs) <= 160 * 1024, "one workgroup per CU");

__device__ inline uint2 lds_ld2(const uint2* base, uint32_t byte_off) {
    return *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ inline void lds_st2(uint2* base, uint32_t byte_off, uint2 v) {
    *reinterpret_cast<uint2*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Loads of a row wavefront for one phase: the pixels of step 1's row and the
// c records of step 3's output row.
struct WsRowIn {
    uint4 ref[kSeg];
    uint4 par[kWsSlices][kSeg];
    uint4 c3[kSeg];
};

// Loads of a column thread for one phase: the b records of step 2's rows.
struct WsColIn {
    uint4 b2[kAggK];
};

struct WsRowLane {
    uint32_t img[kSeg], col4[kSeg], par[kWsSlices][kSeg], inval[kSeg], cbs[kSeg], vout[kSeg], recw;
    bool pok[kWsSlices][kSeg];
};

// Row wavefront: loads for phase p (step 1 of chunk p, step 3 of chunk p - 2).
// kFused: the pixels of both views for the raw cost; else the two slices'
// raw costs of the row from the cost volume (in the x words of in.par).
template <bool kFused>
__device__ inline void ws_row_load(const AggArgs& A, int ys, int p, int w, const WsRowLane& ln,
                                   const AggRes& R, WsRowIn& in) {
    const uint32_t W = (uint32_t)A.W, Wp = (uint32_t)A.rec.Wp;
    const uint32_t yq = (uint32_t)min(ys + kAggK * p + w, A.H - 1);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        if constexpr (kFused) {
            in.ref[j] = ld128(R.rIr, ln.img[j], yq * W * 16);
#pragma unroll
            for (int s = 0; s < kWsSlices; ++s)
                in.par[s][j] = ld128(R.rIp, ln.par[s][j], yq * W * 16);
        } else {
#pragma unroll
            for (int s = 0; s < kWsSlices; ++s)
                in.par[s][j].x = ld32(R.rq, ln.col4[j], yq * W * 4 + s * R.in_slice_bytes);
        }
    }
    const int y2 = ys + kAggK * (p - 2) + w - 2 * kLMax - 1;
    const uint32_t rc = (uint32_t)(y2 >= 0 && y2 < A.H ? y2 : A.H);
#pragma unroll
    for (int j = 0; j < kSeg; ++j) in.c3[j] = ld128(R.rC, ln.recw * 4 + 1024 * j, rc * Wp * 16);
}

// Column thread: loads for step 2 of chunk q (b rows ys + kAggK q + k).
__device__ inline void ws_col_load(const AggArgs& A, int ys, int q, uint32_t reco,
                                   const AggRes& R, WsColIn& in) {
    const uint32_t Wp = (uint32_t)A.rec.Wp;
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint32_t rb = (uint32_t)min(ys + kAggK * q + k, A.H + kLMax);
        in.b2[k] = ld128(R.rB, reco * 4, rb * Wp * 16);
    }
}

// Inclusive row prefixes of the two rows of 256 values the wavefront holds
// in segment layout (lane l, segment j: column 64 j + l), written to its own
// LDS row as P(c) at index c + kWsP0.  The values pass through that row so
// that lane l takes the four consecutive columns 4 l .. 4 l + 3: it adds them
// up in order, one wavefront scan of the lane totals (DPP row shifts 1, 2, 4,
// 8 and row broadcasts 15 and 31) gives each lane the sum of the columns
// before its four, and the prefixes go back as two 16-byte stores.  Sums are
// mod 2^32; only differences of them are used.
__device__ inline void ws_scan_row(const uint32_t (&v)[kWsSlices][kSeg], uint2* row) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) row[64 * j + lane + kWsP0] = make_uint2(v[0][j], v[1][j]);
    __builtin_amdgcn_wave_barrier();  // the row is this wavefront's own
    uint32_t a[kWsSlices][4];
    uint4 lo, hi;  // columns 4 l, 4 l + 1 and 4 l + 2, 4 l + 3, both slices each
    __builtin_memcpy(&lo, __builtin_assume_aligned(row + kWsP0 + 4 * lane, 16), 16);
    __builtin_memcpy(&hi, __builtin_assume_aligned(row + kWsP0 + 4 * lane + 2, 16), 16);
    a[0][0] = lo.x, a[1][0] = lo.y, a[0][1] = lo.z, a[1][1] = lo.w;
    a[0][2] = hi.x, a[1][2] = hi.y, a[0][3] = hi.z, a[1][3] = hi.w;
    uint32_t tot[kWsSlices];
#pragma unroll
    for (int s = 0; s < kWsSlices; ++s) {
        a[s][1] += a[s][0];
        a[s][2] += a[s][1];
        a[s][3] += a[s][2];
        tot[s] = a[s][3];
    }
#define DCO_WS_SCAN(CTRL, MASK) \
    _Pragma("unroll") for (int s = 0; s < kWsSlices; ++s) tot[s] += dpp<CTRL, MASK>(tot[s]);
    DCO_WS_SCAN(0x111, 0xf)
    DCO_WS_SCAN(0x112, 0xf)
    DCO_WS_SCAN(0x114, 0xf)
    DCO_WS_SCAN(0x118, 0xf)
    DCO_WS_SCAN(0x142, 0xa)
    DCO_WS_SCAN(0x143, 0xc)
#undef DCO_WS_SCAN
#pragma unroll
    for (int s = 0; s < kWsSlices; ++s) {
        const uint32_t before = tot[s] - a[s][3];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[s][i] += before;
    }
    lo = make_uint4(a[0][0], a[1][0], a[0][1], a[1][1]);
    hi = make_uint4(a[0][2], a[1][2], a[0][3], a[1][3]);
    __builtin_memcpy(__builtin_assume_aligned(row + kWsP0 + 4 * lane, 16), &lo, 16);
    __builtin_memcpy(__builtin_assume_aligned(row + kWsP0 + 4 * lane + 2, 16), &hi, 16);
    __builtin_amdgcn_wave_barrier();
}

// Row wavefront w, phase p: step 3 of chunk p - 2 and step 1 of chunk p.
template <bool kFused>
__device__ inline void ws_row_phase(const AggArgs& A, int ys, int y0, int y1, int p, int w,
                                    const WsRowLane& ln, const AggRes& R, const WsRowIn& in,
                                    AggLdsWs& S) {
    // Both steps run as one straight block so that their LDS round trips
    // overlap; in the phases where a step has no chunk its LDS writes land in
    // rows nobody reads and its stores are skipped.
    const int lane = threadIdx.x & 63;
    const int W = A.W;
    uint2* row = S.prow[p & 1][w];
    // step 3 of chunk p - 2: vertical range sums of ring 2 (E2)
    uint32_t e2[kWsSlices][kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const uint32_t o = in.c3[j].x;  // ring 2 offsets in 8-byte words
        const uint2 a = S.ring2[ln.cbs[j] + (o & 0xffff)], b = S.ring2[ln.cbs[j] + (o >> 16)];
        e2[0][j] = a.x - b.x;
        e2[1][j] = a.y - b.y;
    }
    // step 1 of chunk p: raw costs of Eq. 1.  Rows below the image load row
    // H - 1 and are not masked: prefixes are modular and every range of a
    // stored output ends inside the image (arms stop at the border), so those
    // rows only change prefixes past the last row any stored output reads.
    uint32_t q[kWsSlices][kSeg];
    if constexpr (!kFused) {
        // the volume holds q 2^-20 exactly (1.0 where the partner is outside
        // the image); columns outside the image load 0
#pragma unroll
        for (int j = 0; j < kSeg; ++j)
#pragma unroll
            for (int s = 0; s < kWsSlices; ++s)
                q[s][j] = (uint32_t)(__builtin_bit_cast(float, in.par[s][j].x) * 0x1p20f);
    } else {
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const uint64_t rc = (uint64_t)in.ref[j].y << 32 | in.ref[j].x;
        const float2 ab = *reinterpret_cast<const float2*>(
            reinterpret_cast<const char*>(S.ab) + in.ref[j].w);
#pragma unroll
        for (int s = 0; s < kWsSlices; ++s) {
            const uint32_t sad = __builtin_amdgcn_sad_u8(in.ref[j].z, in.par[s][j].z, 0u);
            const uint64_t x = rc ^ ((uint64_t)in.par[s][j].y << 32 | in.par[s][j].x);
            const uint32_t h = (uint32_t)__popcll(x);
            q[s][j] = q20_term(ab.x, S.tabA[sad]) + q20_term(ab.y, S.tabC[h]);
        }
    }
    // every lookup stays unconditional; the selects are lane-mask cndmasks
    asm volatile(""
                 : "+v"(q[0][0]), "+v"(q[0][1]), "+v"(q[0][2]), "+v"(q[0][3]), "+v"(q[1][0]),
                   "+v"(q[1][1]), "+v"(q[1][2]), "+v"(q[1][3]));
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
#pragma unroll
        for (int s = 0; s < kWsSlices; ++s) q[s][j] = ln.pok[s][j] ? q[s][j] : ln.inval[j];
    }
    // step 3: row prefixes of E2 in this wavefront's row, then the horizontal
    // range sums and the final division
    ws_scan_row(e2, row);
    float out[kWsSlices][kSeg];
    const uint32_t pbw = (uint32_t)(lane + kWsP0 - 1) * 8;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const uint32_t lr = in.c3[j].z;  // arm offsets in 8-byte words
        const uint2 a = lds_ld2(row, pbw + 512 * j + (lr & 0xff));
        const uint2 b = lds_ld2(row, pbw + 512 * j - ((lr >> 8) & 0xff));
        const float nf = __builtin_bit_cast(float, in.c3[j].w);
        const float rcp = __builtin_bit_cast(float, in.c3[j].y);
        out[0][j] = div_q20(a.x - b.x, nf, rcp);
        out[1][j] = div_q20(a.y - b.y, nf, rcp);
    }
    // step 1: its row prefixes replace step 3's in the same row (LDS keeps
    // this wavefront's order, so step 3's reads above see the old values)
    ws_scan_row(q, row);
    const int y2 = ys + kAggK * (p - 2) + w - 2 * kLMax - 1;
    if (p >= 2 && y2 >= y0 && y2 < y1) {  // uniform
        if (R.paired && R.nout == kWsSlices) {  // uniform: the pair's minimum first
            // div_q20 of an unsigned sum is never negative nor -0, so the bits
            // order like the values, and bit 31 of b1 - b0 is set exactly when
            // b1 < b0 (the second slice strictly smaller)
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                const uint32_t b0 = __builtin_bit_cast(uint32_t, out[0][j]);
                const uint32_t b1 = __builtin_bit_cast(uint32_t, out[1][j]);
                out[0][j] = __builtin_bit_cast(float, ((b1 - b0) & 0x80000000u) | min(b0, b1));
                out[1][j] = __builtin_bit_cast(float, max(b0, b1));
            }
        }
#pragma unroll
        for (int s = 0; s < kWsSlices; ++s)
            if (s < R.nout)  // uniform
#pragma unroll
                for (int j = 0; j < kSeg; ++j)
                    st32(out[s][j], R.rOut, ln.vout[j], (uint32_t)(y2 * W) * 4 + s * R.slice_bytes);
    }
}

// Column thread ct (its column's ring byte offset cb), step 2 of chunk q.
__device__ inline void ws_col_phase(int q, int nch, int ct, uint32_t cb, const WsColIn& in,
                                    uint32_t (&cp1)[kWsSlices], uint32_t (&cp2)[kWsSlices],
                                    uint32_t& off1, uint32_t& off2, AggLdsWs& S) {
    if (q >= nch) return;  // uniform
    const uint2* rows = S.prow[q & 1][0];
    uint32_t e1[kWsSlices][kAggK];
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint32_t a = in.b2[k].z;  // arm offsets in 8-byte words
        const uint32_t pb = (uint32_t)(k * kWsPStride + ct + kWsP0 - 1) * 8;
        const uint2 hi = lds_ld2(rows, pb + (a & 0xff)), lo = lds_ld2(rows, pb - ((a >> 8) & 0xff));
        e1[0][k] = hi.x - lo.x;
        e1[1][k] = hi.y - lo.y;
    }
    // push a row, then read that row's range, before the next push
    uint32_t s1[kWsSlices][kAggK];
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        cp1[0] += e1[0][k];
        cp1[1] += e1[1][k];
        lds_st2(S.ring1, cb + off1, make_uint2(cp1[0], cp1[1]));
        const uint32_t r = in.b2[k].y;  // ring 1 offsets in bytes
        const uint2 hi = lds_ld2(S.ring1, cb + (r & 0xffff)), lo = lds_ld2(S.ring1, cb + (r >> 16));
        s1[0][k] = hi.x - lo.x;
        s1[1][k] = hi.y - lo.y;
        off1 = off1 + kWsSlotBytes == kWsRing1 * kWsSlotBytes ? 0u : off1 + kWsSlotBytes;
    }
#pragma unroll
    for (int k = 0; k < kAggK; ++k) {
        const uint4 b = in.b2[k];
        const uint32_t half = (b.z >> 16) & 1023, sh = b.z >> 26;
#pragma unroll
        for (int s = 0; s < kWsSlices; ++s) {
            const uint64_t n = (uint64_t)(s1[s][k] + half) * b.x;
            cp2[s] += (uint32_t)(n >> sh);
        }
        lds_st2(S.ring2, cb + off2, make_uint2(cp2[0], cp2[1]));
        off2 = off2 + kWsSlotBytes == kWsRing2 * kWsSlotBytes ? 0u : off2 + kWsSlotBytes;
    }
}

// Output rows [y0, y1) of slices d and d + 1 and column strip `strip`
// (512 threads; two stages); slices at or past dend are computed but not
// stored.  kFused: the raw cost computed from the packed pixels; else read
// from the cost volume A.cost.  The records must be written with kRecWs.
template <bool kFused = true>
__device__ inline void agg_stream_ws(const AggArgs& A, int d, int dend, int strip, int y0, int y1,
                                     AggLdsWs& S) {
    const int W = A.W, H = A.H;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int x0 = strip * kStripOut;
    const size_t slice = (size_t)W * H;

    if constexpr (kFused) {
        for (int i = t; i < 766; i += kWsThreads) S.tabA[i] = A.tabA[i];
        if (t < 65) S.tabC[t] = A.tabC[t];
        if (t <= kLMax) {
            const int L = min(t, A.L1);
            S.ab[t] = make_float2(A.alpha[L], A.beta[L]);
        }
    }
    if (t < 2 * kAggK * kWsP0) {  // P(-1) and the entries before it, every row
        const int r = t / kWsP0;
        S.prow[r / kAggK][r % kAggK][t % kWsP0] = make_uint2(0u, 0u);
    }
    // zero column prefixes: rows before the start contribute nothing
    for (int i = t; i < kWsRing1 * kRingStride; i += kWsThreads) S.ring1[i] = make_uint2(0u, 0u);
    for (int i = t; i < kWsRing2 * kRingStride; i += kWsThreads) S.ring2[i] = make_uint2(0u, 0u);

    const uint32_t P4 = (uint32_t)(slice * 4);
    AggRes R;
    const uint4* Iref = A.ref == 0 ? A.pixL : A.pixR;
    const uint4* Ipar = A.ref == 0 ? A.pixR : A.pixL;
    R.rB = make_rsrc(A.rec.b, (uint32_t)(A.rec.Wp * (H + kLMax + 1)) * 16);
    R.rC = make_rsrc(A.rec.c, (uint32_t)(A.rec.Wp * (H + 1)) * 16);
    R.rIr = make_rsrc(Iref, 4 * P4);
    R.rIp = make_rsrc(Ipar, 4 * P4);
    const int nout = min(kWsSlices, min(A.D, dend) - d);  // slices to store
    // raw costs of slices d and d + 1; past the last slice, slice d again
    R.rq = kFused ? R.rB
                  : make_rsrc(A.cost + (size_t)d * slice, (uint32_t)min(kWsSlices, A.D - d) * P4);
    R.in_slice_bytes = A.D - d >= 2 ? P4 : 0u;
    R.rOut = make_rsrc(A.out + (size_t)d * slice, (uint32_t)nout * P4);
    R.slice_bytes = P4;
    R.nout = nout;
    R.paired = A.paired;

    const int warm = 2 * kLMax + 1;
    const int ys = max(0, y0 - warm);
    const int nch = (y1 + warm - ys + kAggK - 1) / kAggK;
    const int last = nch + 1;  // phases 0 .. nch + 1
    __syncthreads();

    if (w < kAggK) {  // row wavefronts
        // the row wavefronts carry the longer chain of each phase; issuing
        // their instructions first when both kinds are ready helps slightly
        __builtin_amdgcn_s_setprio(1);
        WsRowLane ln;
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const int i = 64 * j + lane;            // strip column of segment j
            const int c = x0 - 2 * kLMax + i;       // image column
            const bool in_img = c >= 0 && c < W;
            ln.img[j] = in_img ? (uint32_t)c * 16 : kOOB;
            ln.col4[j] = in_img ? (uint32_t)c * 4 : kOOB;
#pragma unroll
            for (int s = 0; s < kWsSlices; ++s) {
                const int cp = A.ref == 0 ? c - d - s : c + d + s;
                const bool pok = in_img && cp >= 0 && cp < W;
                ln.par[s][j] = pok ? (uint32_t)cp * 16 : kOOB;
                ln.pok[s][j] = pok;
            }
            ln.inval[j] = in_img ? (1u << 20) : 0u;
            // ring-2 column (kRingCols + 1, never written, for columns without one)
            const bool rok = i >= kLMax && i < kLMax + kRingCols;
            ln.cbs[j] = (uint32_t)(rok ? i - kLMax : kRingCols + 1);
            ln.vout[j] =
                i >= 2 * kLMax && i < 2 * kLMax + kStripOut && c < W ? (uint32_t)c * 4 : kOOB;
        }
        ln.recw = (uint32_t)(x0 - 2 * kLMax + lane + A.rec.apron) * 4;
        WsRowIn ia, ib;
        ws_row_load<kFused>(A, ys, 0, w, ln, R, ia);
        for (int p = 0;; p += 2) {
            ws_row_load<kFused>(A, ys, p + 1, w, ln, R, ib);
            ws_row_phase<kFused>(A, ys, y0, y1, p, w, ln, R, ia, S);
            __syncthreads();
            if (p + 1 > last) break;
            ws_row_load<kFused>(A, ys, p + 2, w, ln, R, ia);
            ws_row_phase<kFused>(A, ys, y0, y1, p + 1, w, ln, R, ib, S);
            __syncthreads();
            if (p + 2 > last) break;
        }
    } else {  // column threads
        const int ct = t - kStripThreads;
        const int c = x0 - 2 * kLMax + ct;
        const int jj = ct - kLMax;
        // threads without a ring column share one scratch column; column
        // kRingCols + 1 stays zero
        const uint32_t cb = (uint32_t)(jj >= 0 && jj < kRingCols ? jj : kRingCols) * 8;
        const uint32_t reco = (uint32_t)(c + A.rec.apron) * 4;
        uint32_t cp1[kWsSlices] = {0, 0}, cp2[kWsSlices] = {0, 0};
        uint32_t off1 = ring_slot(ys, kWsRing1) * kWsSlotBytes;
        uint32_t off2 = ring_slot(ys - kLMax, kWsRing2) * kWsSlotBytes;
        WsColIn ja, jb;
        ws_col_load(A, ys, 0, reco, R, ja);
        __syncthreads();  // phase 0: no step 2 yet
        for (int p = 1;; p += 2) {
            if (p > last) break;
            ws_col_load(A, ys, p, reco, R, jb);
            ws_col_phase(p - 1, nch, ct, cb, ja, cp1, cp2, off1, off2, S);
            __syncthreads();
            if (p + 1 > last) break;
            ws_col_load(A, ys, p + 1, reco, R, ja);
            ws_col_phase(p, nch, ct, cb, jb, cp1, cp2, off1, off2, S);
            __syncthreads();
        }
    }
}

// Work item of block b of n, remapped so that the blocks one XCD runs
// (round-robin block -> XCD dispatch) get consecutive items, which then
// share their inputs in that XCD's L2.
__device__ inline int xcd_work_item(int b, int n) {
    const int xcd = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

// ===========================================================================
// Winner-take-all (Eq. 3) with parabola sub-pixel refinement; LR check
// ===========================================================================

// Parabola vertex offset through (d-1, m), (d, c), (d+1, pl), in this FP32
// order, clamped to [-0.5, 0.5]; 0 at the range ends or for den <= 0.
__device__ inline float subpixel_delta(float m, float c, float pl, int bd, int D) {
    float del = 0.f;
    if (bd > 0 && bd < D - 1) {
        const float num = m - pl;
        const float den = (m - c) + (pl - c);
        if (den > 0.f) {
            del = num / (2.0f * den);
            del = fminf(fmaxf(del, -0.5f), 0.5f);
        }
    }
    return del;
}


// Pixel i of a D-slice volume: smallest d minimising agg, with the values at
// d - 1 and d + 1 tracked on the fly (ties keep the smallest d).
__device__ inline void wta_pixel(const float* __restrict__ agg, int P, int D, int i,
                                 int subpixel, int16_t* dout, float* delta_out) {
    float best = agg[i], prev = best, m = 0.f, pl = 0.f;
    int bd = 0;
    constexpr int U = 8;
    int d = 1;
    for (; d + U <= D; d += U) {
        float v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = agg[(size_t)(d + k) * P + i];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (d + k == bd + 1) pl = v[k];
            if (v[k] < best) {
                best = v[k];
                bd = d + k;
                m = prev;
            }
            prev = v[k];
        }
    }
    for (; d < D; ++d) {
        const float v = agg[(size_t)d * P + i];
        if (d == bd + 1) pl = v;
        if (v < best) {
            best = v;
            bd = d;
            m = prev;
        }
        prev = v;
    }
    *dout = (int16_t)bd;
    if (delta_out) *delta_out = subpixel ? subpixel_delta(m, best, pl, bd, D) : 0.f;
}

// Four consecutive pixels i4 .. i4 + 3 of a D-slice volume (P % 4 == 0, so
// every slice row of four is 16-byte aligned): the same rule as wta_pixel
// per component, with one 16-byte load per slice and eight slices in flight.
__device__ inline void wta_quad_step(float v, int d, float& best, int& bd, float& m, float& pl,
                                     float& prev) {
    if (d == bd + 1) pl = v;
    if (v < best) {
        best = v;
        bd = d;
        m = prev;
    }
    prev = v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline void wta_quad(const float* __restrict__ agg, int P, int D, int i4, int subpixel,
                                int16_t* __restrict__ dout, float* __restrict__ delta_out) {
    // each volume is read once: non-temporal loads keep it from evicting
    // reused data from the caches
    const f32x4* __restrict__ a4 = reinterpret_cast<const f32x4*>(agg + i4);
    const size_t s4 = (size_t)P / 4;
    const f32x4 v0 = __builtin_nontemporal_load(a4);
    float best[4] = {v0.x, v0.y, v0.z, v0.w}, prev[4] = {v0.x, v0.y, v0.z, v0.w};
    float m[4] = {0.f, 0.f, 0.f, 0.f}, pl[4] = {0.f, 0.f, 0.f, 0.f};
    int bd[4] = {0, 0, 0, 0};
    constexpr int U = 8;
    int d = 1;
    for (; d + U <= D; d += U) {
        f32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(a4 + (size_t)(d + k) * s4);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            wta_quad_step(v[k].x, d + k, best[0], bd[0], m[0], pl[0], prev[0]);
            wta_quad_step(v[k].y, d + k, best[1], bd[1], m[1], pl[1], prev[1]);
            wta_quad_step(v[k].z, d + k, best[2], bd[2], m[2], pl[2], prev[2]);
            wta_quad_step(v[k].w, d + k, best[3], bd[3], m[3], pl[3], prev[3]);
        }
    }
    for (; d < D; ++d) {
        const f32x4 v = __builtin_nontemporal_load(a4 + (size_t)d * s4);
        wta_quad_step(v.x, d, best[0], bd[0], m[0], pl[0], prev[0]);
        wta_quad_step(v.y, d, best[1], bd[1], m[1], pl[1], prev[1]);
        wta_quad_step(v.z, d, best[2], bd[2], m[2], pl[2], prev[2]);
        wta_quad_step(v.w, d, best[3], bd[3], m[3], pl[3], prev[3]);
    }
    const uint32_t lo = (uint32_t)(uint16_t)bd[0] | (uint32_t)(uint16_t)bd[1] << 16;
    const uint32_t hi = (uint32_t)(uint16_t)bd[2] | (uint32_t)(uint16_t)bd[3] << 16;
    *reinterpret_cast<uint2*>(dout + i4) = make_uint2(lo, hi);
    if (delta_out) {
        float4 del = make_float4(0.f, 0.f, 0.f, 0.f);
        if (subpixel) {
            del.x = subpixel_delta(m[0], best[0], pl[0], bd[0], D);
            del.y = subpixel_delta(m[1], best[1], pl[1], bd[1], D);
            del.z = subpixel_delta(m[2], best[2], pl[2], bd[2], D);
            del.w = subpixel_delta(m[3], best[3], pl[3], bd[3], D);
        }
        *reinterpret_cast<float4*>(delta_out + i4) = del;
    }
}

// Winner-take-all on a volume in the paired layout: the same rule and the
// same result as wta_pixel / wta_quad, since each even slice holds the
// smaller cost of its pair (the first on a tie) and the pairs are visited in
// order with a strict comparison; only the G = ceil(D / 2) even slices are
// read.  The sub-pixel step gathers the costs at d - 1 and d + 1, which is
// exactly where wta_pixel's m and pl come from when 0 < d < D - 1 (the only
// case in which subpixel_delta uses them).
__device__ inline void wta_pair_step(uint32_t s, int g, float& best, int& bd) {
    const float v = __builtin_bit_cast(float, s & 0x7fffffffu);
    if (v < best) {
        best = v;
        bd = 2 * g + (int)(s >> 31);
    }
}

__device__ inline float wta_pair_delta(const float* __restrict__ vol, int P, int D, int i,
                                       float best, int bd) {
    if (bd <= 0 || bd >= D - 1) return 0.f;
    return subpixel_delta(paired_at(vol, P, D, bd - 1, i), best, paired_at(vol, P, D, bd + 1, i),
                          bd, D);
}

__device__ inline void wta_pairs_pixel(const float* __restrict__ vol, int P, int D, int i,
                                       int subpixel, int16_t* dout, float* delta_out) {
    const uint32_t* __restrict__ u = reinterpret_cast<const uint32_t*>(vol);
    const int G = (D + 1) / 2;
    float best = __builtin_bit_cast(float, u[i] & 0x7fffffffu);
    int bd = (int)(u[i] >> 31);
    for (int g = 1; g < G; ++g) wta_pair_step(u[(size_t)2 * g * P + i], g, best, bd);
    *dout = (int16_t)bd;
    if (delta_out) *delta_out = subpixel ? wta_pair_delta(vol, P, D, i, best, bd) : 0.f;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pair step that also keeps, for the left view's parabola, the word of the
// pair before the best one (prevw) and of the pair after it (nextw): the
// neighbour of the winner in an adjacent pair is then often that pair's
// minimum, already loaded.
__device__ inline void wta_pair_step_tr(uint32_t s, int g, float& best, int& bd, uint32_t& lastw,
                                        uint32_t& prevw, uint32_t& nextw, bool& pend) {
    const float v = __builtin_bit_cast(float, s & 0x7fffffffu);
    if (pend) {
        nextw = s;
        pend = false;
    }
    if (v < best) {
        best = v;
        bd = 2 * g + (int)(s >> 31);
        prevw = lastw;
        pend = true;
    }
    lastw = s;
}

// wta_pair_delta with the adjacent pairs' words from the scan: the winner's
// pair partner is that pair's maximum (the odd slice), and the neighbour in
// the adjacent pair is read only when it is not that pair's minimum.  The
// values are the same ones paired_at decodes.
__device__ inline float wta_pair_delta_tr(const float* __restrict__ vol, int P, int D, int i,
                                          float best, int bd, uint32_t prevw, uint32_t nextw) {
    if (bd <= 0 || bd >= D - 1) return 0.f;
    const int g = bd >> 1;
    const float partner = vol[(size_t)(2 * g + 1) * P + i];
    float m, pl;
    if ((bd & 1) == 0) {
        m = (prevw >> 31) ? __builtin_bit_cast(float, prevw & 0x7fffffffu)
                          : vol[(size_t)(2 * g - 1) * P + i];
        pl = partner;
    } else {
        m = partner;
        pl = (nextw >> 31) == 0u || 2 * g + 3 >= D ? __builtin_bit_cast(float, nextw & 0x7fffffffu)
                                                   : vol[(size_t)(2 * g + 3) * P + i];
    }
    return subpixel_delta(m, best, pl, bd, D);
}

// Four consecutive pixels (P % 4 == 0): one 16-byte load per even slice,
// 21 slices in flight.  kSub: the left view, with the parabola's offset
// into delta_out; else delta_out is null.
template <bool kSub>
__device__ inline void wta_pairs_quad(const float* __restrict__ vol, int P, int D, int i4,
                                      int subpixel, int16_t* __restrict__ dout,
                                      float* __restrict__ delta_out) {
    const int G = (D + 1) / 2;
    const u32x4* __restrict__ s4 = reinterpret_cast<const u32x4*>(vol + i4);
    const size_t st = (size_t)P / 2;  // two slices, in 16-byte words
    const u32x4 w0 = __builtin_nontemporal_load(s4);
    const uint32_t w0s[4] = {w0.x, w0.y, w0.z, w0.w};
    float best[4];
    int bd[4];
    uint32_t lastw[4], prevw[4] = {0u, 0u, 0u, 0u}, nextw[4] = {0u, 0u, 0u, 0u};
    bool pend[4] = {true, true, true, true};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        best[q] = __builtin_bit_cast(float, w0s[q] & 0x7fffffffu);
        bd[q] = (int)(w0s[q] >> 31);
        lastw[q] = w0s[q];
    }
    const auto step = [&](const u32x4& v, int g) {
        const uint32_t vs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (kSub)
                wta_pair_step_tr(vs[q], g, best[q], bd[q], lastw[q], prevw[q], nextw[q], pend[q]);
            else
                wta_pair_step(vs[q], g, best[q], bd[q]);
        }
    };
    constexpr int U = 21;  // 21 loads in flight per thread (three batches for D = 128)
    int g = 1;
    for (; g + U <= G; g += U) {
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(s4 + (size_t)(g + k) * st);
#pragma unroll
        for (int k = 0; k < U; ++k) step(v[k], g + k);
    }
    if (g < G) {  // the last groups as one batch (loads clamped to the last group)
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = __builtin_nontemporal_load(s4 + (size_t)min(g + k, G - 1) * st);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (g + k < G) step(v[k], g + k);
    }
    const uint32_t lo = (uint32_t)(uint16_t)bd[0] | (uint32_t)(uint16_t)bd[1] << 16;
    const uint32_t hi = (uint32_t)(uint16_t)bd[2] | (uint32_t)(uint16_t)bd[3] << 16;
    *reinterpret_cast<uint2*>(dout + i4) = make_uint2(lo, hi);
    if constexpr (kSub) {
        float del[4] = {0.f, 0.f, 0.f, 0.f};
        if (subpixel) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                del[q] = wta_pair_delta_tr(vol, P, D, i4 + q, best[q], bd[q], prevw[q], nextw[q]);
        }
        *reinterpret_cast<float4*>(delta_out + i4) = make_float4(del[0], del[1], del[2], del[3]);
    }
}

__device__ inline void lr_pixel(const int16_t* __restrict__ dL, const float* __restrict__ deltaL,
                                const int16_t* __restrict__ dR, int W, int x, int y, int maxdiff,
                                float* __restrict__ disp, uint8_t* __restrict__ valid) {
    const size_t i = (size_t)y * W + x;
    const int dl = dL[i];
    const int xr = x - dl;
    const bool ok = xr >= 0 && abs(dl - (int)dR[(size_t)y * W + xr]) <= maxdiff;
    valid[i] = ok ? 1 : 0;
    disp[i] = ok ? (float)dl + deltaL[i] : 0.0f;
}

}  // namespace dco
