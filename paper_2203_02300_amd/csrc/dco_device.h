// dco_device.h -- device-side bodies of every stage of the plain matcher.
//
// The one-call kernels (k_census.hip, k_aggregate.hip, k_wta.hip) and the
// persistent batched kernel (k_batch.hip) run exactly these functions, so a
// pair matched alone and the same pair matched in a batch give the same bits.
// Each function takes its LDS as an explicit struct so the persistent kernel
// can overlay the stages' LDS in one union.
#pragma once

#include "dco_internal.h"

namespace dco {

// ===========================================================================
// Census codes and cross-support arms (Sec. 4.1; C_census of Eq. 1)
// ===========================================================================

constexpr int kCenTW = 64, kCenTH = 16;                                  // pixel tile
constexpr int kCenRW = kCenTW + 2 * kLMax, kCenRH = kCenTH + 2 * kLMax;  // staged RGB region
constexpr int kCenHW = 4, kCenHH = 4;                                     // census half-window limits
constexpr int kCenGW = kCenTW + 2 * kCenHW, kCenGH = kCenTH + 2 * kCenHH;

struct CensusLds {
    uint32_t rgb[kCenRH][kCenRW];
    uint32_t grey[kCenGH][kCenGW];
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline uint32_t grey_of(uint32_t c) {
    uint32_t r = c & 0xffu, g = (c >> 8) & 0xffu, b = (c >> 16) & 0xffu;
    return (77u * r + 150u * g + 29u * b + 128u) >> 8;
}

// Largest per-channel absolute difference below tau?
__device__ inline bool close_rgb(uint32_t a, uint32_t b, int tau) {
    int dr = (int)(a & 0xffu) - (int)(b & 0xffu);
    int dg = (int)((a >> 8) & 0xffu) - (int)((b >> 8) & 0xffu);
    int db = (int)((a >> 16) & 0xffu) - (int)((b >> 16) & 0xffu);
    int m = max(max(abs(dr), abs(dg)), abs(db));
    return m < tau;
}

// One 64 x 16 tile at (x0, y0), 256 threads.  The tile plus a kLMax apron
// (edge-clamped) is staged in LDS as packed RGB words; grey levels of the
// tile plus the census apron go to a second array.
//   grey:   Y = (77 R + 150 G + 29 B + 128) >> 8
//   census: bit k = Y(q_k) < Y(p), neighbours row-major without the centre
//   arms:   steps j = 1.. while inside, j <= L1 and max channel |diff| < tau1
__device__ inline void census_tile(const uint8_t* __restrict__ rgb, int W, int H, int cw, int ch,
                                   int L1, int tau1, uint64_t* __restrict__ census,
                                   uint32_t* __restrict__ arms, uint32_t* __restrict__ rgb_packed,
                                   int x0, int y0, CensusLds& S) {
    const int t = threadIdx.x;
    for (int i = t; i < kCenRW * kCenRH; i += 256) {
        int ry = i / kCenRW, rx = i - ry * kCenRW;
        int gx = clampi(x0 - kLMax + rx, 0, W - 1), gy = clampi(y0 - kLMax + ry, 0, H - 1);
        const uint8_t* p = rgb + 3 * ((size_t)gy * W + gx);
        S.rgb[ry][rx] = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
    }
    __syncthreads();
    for (int i = t; i < kCenGW * kCenGH; i += 256) {
        int gy = i / kCenGW, gx = i - gy * kCenGW;
        S.grey[gy][gx] = grey_of(S.rgb[gy + kLMax - kCenHH][gx + kLMax - kCenHW]);
    }
    __syncthreads();

    const int hw = cw >> 1, hh = ch >> 1;
    const int tx = t & 63;
    for (int k = 0; k < kCenTH / 4; ++k) {
        const int ty = (t >> 6) + 4 * k;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H) continue;
        const uint32_t c = S.grey[ty + kCenHH][tx + kCenHW];
        uint64_t code = 0;
        int bit = 0;
        for (int dy = -hh; dy <= hh; ++dy) {
            for (int dx = -hw; dx <= hw; ++dx) {
                if (dy == 0 && dx == 0) continue;
                uint32_t v = S.grey[ty + kCenHH + dy][tx + kCenHW + dx];
                code |= (uint64_t)(v < c) << bit;
                ++bit;
            }
        }
        census[(size_t)y * W + x] = code;

        const int rx = tx + kLMax, ry = ty + kLMax;
        const uint32_t cp = S.rgb[ry][rx];
        if (rgb_packed) rgb_packed[(size_t)y * W + x] = cp;
        int al = 0, ar = 0, au = 0, ad = 0;
        const int ml = min(L1, x), mr = min(L1, W - 1 - x);
        const int mu = min(L1, y), md = min(L1, H - 1 - y);
        while (al < ml && close_rgb(S.rgb[ry][rx - al - 1], cp, tau1)) ++al;
        while (ar < mr && close_rgb(S.rgb[ry][rx + ar + 1], cp, tau1)) ++ar;
        while (au < mu && close_rgb(S.rgb[ry - au - 1][rx], cp, tau1)) ++au;
        while (ad < md && close_rgb(S.rgb[ry + ad + 1][rx], cp, tau1)) ++ad;
        arms[(size_t)y * W + x] =
            (uint32_t)al | ((uint32_t)ar << 8) | ((uint32_t)au << 16) | ((uint32_t)ad << 24);
    }
}

// ===========================================================================
// Region counts and packed aggregation records of one pixel
// ===========================================================================
//   N1 = sum over y' in [y-u, y+dn] of (l(x,y') + r(x,y') + 1)
//   N2 = sum over x' in [x-l, x+r] of (u(x',y) + dn(x',y) + 1)
// Stage-1 rounding uses sh = 31 + ceil(log2 N1) and m = ceil(2^sh / N1) <
// 2^32, so floor(n / N1) = (n * m) >> sh for every 0 <= n < 2^31 (N1 <= 2^11).
// The final division uses (N, RN(1/N)) with N = N2 (two stages) or N1 (one).
// Record layout: see AggRecords.
__device__ inline void geometry_pixel(const uint32_t* __restrict__ arms, int W, int H, int iters,
                                      const AggRecords& rec, int x, int y) {
    const uint32_t a = arms[(size_t)y * W + x];
    const uint32_t l = a & 0xff, r = (a >> 8) & 0xff, u = (a >> 16) & 0xff, dn = a >> 24;
    uint32_t n1 = 0, n2 = 0;
    // arms from census_tile stay inside the image; the clamps only keep a
    // corrupted arms buffer from reading outside it
    for (int yy = max(0, y - (int)u); yy <= min(H - 1, y + (int)dn); ++yy) {
        uint32_t b = arms[(size_t)yy * W + x];
        n1 += (b & 0xff) + ((b >> 8) & 0xff) + 1;
    }
    for (int xx = max(0, x - (int)l); xx <= min(W - 1, x + (int)r); ++xx) {
        uint32_t b = arms[(size_t)y * W + xx];
        n2 += ((b >> 16) & 0xff) + (b >> 24) + 1;
    }
    const uint32_t lg = n1 <= 1 ? 0u : 32u - (uint32_t)__clz((int)(n1 - 1));
    const uint32_t sh = 31u + lg;
    const uint64_t num = (uint64_t)1 << sh;
    const uint32_t m = (uint32_t)((num + n1 - 1) / n1);
    const uint32_t n = iters == 1 ? n1 : n2;
    const float rcp = 1.0f / (float)n;
    const size_t i = (size_t)y * rec.Wp + x + rec.apron;
    rec.a[i] = a;
    rec.b[i] = make_uint2(m, (n1 >> 1) | (sh << 10) | (u << 16) | (dn << 21));
    rec.c[i] = make_uint2(__float_as_uint(rcp),
                          l | (r << 5) | (u << 10) | (dn << 15) | (n << 20));
}

// ===========================================================================
// Streaming two-stage aggregation (Eq. 2 twice), one slice x one column strip
// ===========================================================================
//
// The strip's 256 threads own 256 consecutive columns: 2 kLMax apron columns
// on each side and kStripOut output columns in the middle.  The workgroup
// streams down the rows; per row
//   H1: E1 = row range sum of q             (block prefix scan + 2 LDS reads)
//   V1: S1 = column range sum of E1         (per-column ring of prefix sums)
//       a1 = floor((S1 + N1/2) / N1)        (exact multiply-shift division)
//   V2: E2 = column range sum of a1         (second per-column ring)
//   H2: S2 = row range sum of E2            (block prefix scan + 2 LDS reads)
//       out = RN(S2 / N2) * 2^-20           (reciprocal + one FMA correction)
// Each ring keeps the last kRing column-prefix rows of one column; only the
// thread owning that column touches it.  Rows come in chunks of kRowChunk
// (four barriers per chunk) and the next chunk's loads are issued before the
// current chunk is processed.  V1 finalises row y - kLMax and H2 row
// y - 2 kLMax - 1 while H1 consumes row y.
//
// Per-pixel data comes from the padded records (zero apron, zero row H)
// through buffer loads with a per-lane column offset and a uniform row
// offset, so the chunk body has no address arithmetic and no bounds branches.
//
// Every sum is an integer and differences of prefix sums are taken mod 2^32
// (every true range sum is below 2^31), so the result does not depend on the
// summation order, and a band of output rows [y0, y1) can start from zero
// prefixes 2 kLMax + 1 rows above y0: the rows before the start then shift
// every prefix by the same constant.

constexpr int kRingCols = kStripThreads - 2 * kLMax;  // ring columns used: 222
constexpr int kRingStride = 224;
constexpr int kPB = kStripThreads + 4;                // prefix row stride (P[-1] at 0)
constexpr uint32_t kRingBytes = kRing * kRingStride * 4;
constexpr uint32_t kOOB = 0x7fffffffu;                // buffer offset that reads as 0

template <int ITERS, bool kFused, int K = kRowChunk>
struct AggLds {
    uint32_t ring1[kRing * kRingStride];
    uint32_t ring2[ITERS == 2 ? kRing * kRingStride : 1];
    uint32_t pbuf[K][kPB];
    __attribute__((aligned(16))) uint32_t wsum[2][K][4];
    float tabA[kFused ? 768 : 1];
    float tabC[kFused ? 65 : 1];
    float ab[kFused ? 2 * (kLMax + 1) : 1];
};

typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ inline rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ inline uint32_t ld32(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
__device__ inline uint2 ld64(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <unsigned Ctrl, unsigned RowMask>
__device__ inline uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, false);
}

// Inclusive scans of K rows at once across the 256 threads of the block.
// Within a wavefront: DPP row shifts 1, 2, 4, 8 and the gfx9 row broadcasts
// 15 and 31, issued step-major so that the K rows' steps interleave.  Across
// the four wavefronts: totals through LDS.  Writes P(t) to pb[k][t + 1]
// (pb[k][0] holds 0).  Two barriers; on return every thread sees every row.
template <int K>
__device__ inline void block_scan_rows(uint32_t (&v)[K], uint32_t (*pb)[kPB],
                                       uint32_t (*ws)[4]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x111, 0xf>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x112, 0xf>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x114, 0xf>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x118, 0xf>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x142, 0xa>(v[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += dpp<0x143, 0xc>(v[k]);
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) ws[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint4 s = *reinterpret_cast<const uint4*>(ws[k]);
        uint32_t off = 0;
        if (w > 0) off += s.x;
        if (w > 1) off += s.y;
        if (w > 2) off += s.z;
        pb[k][t + 1] = v[k] + off;
    }
    __syncthreads();
}

// Byte offset inside a ring of the row `back` rows behind the row whose slot
// byte offset is `slot_off` (0 <= back < kRing).  The unsigned minimum picks
// the wrapped value when the subtraction goes below zero.
__device__ inline uint32_t ring_off(uint32_t slot_off, int back) {
    const uint32_t a = slot_off - (uint32_t)back * (kRingStride * 4);
    return min(a, a + kRingBytes);
}

__device__ inline uint32_t lds_ld(const uint32_t* base, uint32_t byte_off) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ inline void lds_st(uint32_t* base, uint32_t byte_off, uint32_t v) {
    *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// RN((float)s / N) given N and RN(1/N).  Exact: q0 = RN(s * y) is within two
// ulps of s/N, r = s - q0 * N is then exact, and s/N is never a float
// midpoint for integer N, so RN(q0 + r * y) = RN(s / N).
__device__ inline float div_rn(uint32_t s, float n, float rcp) {
    const float a = (float)s;
    const float q0 = a * rcp;
    const float r = __builtin_fmaf(-q0, n, a);
    return __builtin_fmaf(r, rcp, q0);
}

struct AggArgs {
    const float* cost;         // staged: D x H x W raw costs
    const uint32_t* rgbL;      // fused: packed RGB of both views (H x W)
    const uint32_t* rgbR;
    const uint64_t* cenL;      // fused: census codes (H x W)
    const uint64_t* cenR;
    const float* tabA;         // fused: Eq. 1 tables
    const float* tabC;
    const float* alpha;
    const float* beta;
    AggRecords rec;            // padded per-pixel records of the reference view
    float* out;                // D x H x W
    int W, H, D, nstrips, ref, L1;
};

// Everything one thread loads for one row step: rows y (H1), y - kLMax (V1)
// and y - 2 kLMax - 1 (V2, H2; row y - kLMax for one stage) of its column.
template <bool kFused>
struct RowData {
    uint32_t q;        // staged: q of row y; fused: 0 or ~0 (row inside the image)
    uint32_t rrgb, prgb;
    uint2 rcen, pcen;  // fused: reference and partner census words
    uint32_t recA;     // arms of row y
    uint2 recB;        // stage-1 division data and vertical arms of row y - kLMax
    uint2 recC;        // final division data and arms of the output row
};

struct Lane {
    uint32_t rec4, rec8;     // record byte offsets of this column (4- and 8-byte records)
    uint32_t img4, img8;     // byte offsets of the clamped column in H x W maps
    uint32_t par4, par8;     // fused: the partner column
    uint32_t col_mask;       // ~0 when the column is inside the image
    uint32_t par_ok;         // ~0 when the partner column is inside the image
};

struct AggRes {
    rsrc_t rA, rB, rC, rq, rIr, rIp, rCr, rCp;
};

template <int ITERS, bool kFused, int K>
__device__ inline void load_rows(const AggArgs& A, int yc, const Lane& ln, const AggRes& R,
                                 RowData<kFused> (&rd)[K]) {
    const int H = A.H;
    const uint32_t Wp = (uint32_t)A.rec.Wp, W = (uint32_t)A.W;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int y = yc + k;
        const int y1 = y - kLMax;
        const int yo = ITERS == 2 ? y - 2 * kLMax - 1 : y1;
        // records: rows outside the image map to the zero row H
        const uint32_t ra = (uint32_t)(y < H ? y : H);
        const uint32_t rb = (uint32_t)(y1 >= 0 && y1 < H ? y1 : H);
        const uint32_t rc = (uint32_t)(yo >= 0 && yo < H ? yo : H);
        rd[k].recA = ld32(R.rA, ln.rec4, ra * Wp * 4);
        rd[k].recB = ld64(R.rB, ln.rec8, rb * Wp * 8);
        rd[k].recC = ld64(R.rC, ln.rec8, rc * Wp * 8);
        const uint32_t yq = (uint32_t)min(y, H - 1);
        const uint32_t row_mask = y < H ? ~0u : 0u;
        if (kFused) {
            rd[k].rrgb = ld32(R.rIr, ln.img4, yq * W * 4);
            rd[k].prgb = ld32(R.rIp, ln.par4, yq * W * 4);
            rd[k].rcen = ld64(R.rCr, ln.img8, yq * W * 8);
            rd[k].pcen = ld64(R.rCp, ln.par8, yq * W * 8);
            rd[k].q = row_mask;
        } else {
            const float v = __builtin_bit_cast(float, ld32(R.rq, ln.img4, yq * W * 4));
            rd[k].q = (uint32_t)(v * 1048576.0f) & row_mask;
        }
    }
}

template <int ITERS, bool kFused, int K>
__device__ inline void process_rows(int yc, int y0, int y1, int W, int c, int t, bool ring_thr,
                                    bool out_thr, const Lane& ln, float* __restrict__ out,
                                    RowData<kFused> (&rd)[K], uint32_t& cp1, uint32_t& cp2,
                                    uint32_t& slot_off, uint32_t* ring1, uint32_t* ring2,
                                    AggLds<ITERS, kFused, K>& S) {
    uint32_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (kFused) {
            const uint32_t a = rd[k].recA;
            const int lmin = min(min((int)(a & 0xff), (int)((a >> 8) & 0xff)),
                                 min((int)((a >> 16) & 0xff), (int)(a >> 24)));
            const uint32_t s = __builtin_amdgcn_sad_u8(rd[k].rrgb, rd[k].prgb, 0u);
            const int h =
                __popc(rd[k].rcen.x ^ rd[k].pcen.x) + __popc(rd[k].rcen.y ^ rd[k].pcen.y);
            const float qa = __builtin_rintf(S.ab[lmin] * S.tabA[s]);
            const float qc = __builtin_rintf(S.ab[kLMax + 1 + lmin] * S.tabC[h]);
            const uint32_t qv = ln.par_ok ? (uint32_t)qa + (uint32_t)qc : (1u << 20);
            v[k] = qv & rd[k].q & ln.col_mask;
        } else {
            v[k] = rd[k].q;
        }
    }
    block_scan_rows<K>(v, S.pbuf, S.wsum[0]);

    uint32_t e2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        {   // H1: E1 of row y = yc + k, pushed as the column prefix of row y
            const uint32_t a = rd[k].recA;
            const int l = a & 0xff, r = (a >> 8) & 0xff;
            const uint32_t e1 = S.pbuf[k][t + r + 1] - S.pbuf[k][t - l];
            cp1 += e1;
            lds_st(ring1, slot_off, cp1);
        }
        if (ITERS == 2) {
            // V2: E2 of row y - 2 kLMax - 1 from the a1 prefix rows: row
            // y2 + dn is 2 kLMax + 1 - dn rows behind y, row y2 - u - 1 shares
            // the slot of row y - u
            const uint32_t g = rd[k].recC.y;
            const int u = (g >> 10) & 31, dn = (g >> 15) & 31;
            const uint32_t e = lds_ld(ring2, ring_off(slot_off, 2 * kLMax + 1 - dn)) -
                               lds_ld(ring2, ring_off(slot_off, u));
            e2[k] = ring_thr ? e : 0u;
        }
        {   // V1: S1 of row yv = y - kLMax (prefix rows yv - u - 1 .. yv + dn)
            const uint32_t g = rd[k].recB.y;
            const int u = (g >> 16) & 31, dn = (g >> 21) & 31;
            const uint32_t s1 = lds_ld(ring1, ring_off(slot_off, kLMax - dn)) -
                                lds_ld(ring1, ring_off(slot_off, kLMax + u + 1));
            if (ITERS == 2) {
                const uint64_t n = (uint64_t)(s1 + (g & 1023));
                cp2 += (uint32_t)((n * rd[k].recB.x) >> ((g >> 10) & 63));
                lds_st(ring2, ring_off(slot_off, kLMax), cp2);
            } else {
                const int yv = yc + k - kLMax;
                const uint32_t gc = rd[k].recC.y;
                const float a1 =
                    div_rn(s1, (float)(gc >> 20), __builtin_bit_cast(float, rd[k].recC.x));
                if (out_thr && yv >= y0 && yv < y1) out[(size_t)yv * W + c] = a1 * 0x1p-20f;
            }
        }
        slot_off = slot_off + kRingStride * 4 == kRingBytes ? 0u : slot_off + kRingStride * 4;
    }
    if (ITERS == 2) {
        block_scan_rows<K>(e2, S.pbuf, S.wsum[1]);
        float a2[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {  // H2: S2 of row y - 2 kLMax - 1
            const uint32_t g = rd[k].recC.y;
            const int l = g & 31, r = (g >> 5) & 31;
            const uint32_t s2 = S.pbuf[k][t + r + 1] - S.pbuf[k][t - l];
            a2[k] = div_rn(s2, (float)(g >> 20), __builtin_bit_cast(float, rd[k].recC.x)) *
                    0x1p-20f;
        }
        if (out_thr) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int y2 = yc + k - 2 * kLMax - 1;
                if (y2 >= y0 && y2 < y1) out[(size_t)y2 * W + c] = a2[k];
            }
        }
    }
}

// Output rows [y0, y1) of slice d and column strip `strip` (256 threads),
// K rows per block-scan round.
template <int ITERS, bool kFused, int K = kRowChunk>
__device__ inline void agg_stream(const AggArgs& A, int d, int strip, int y0, int y1,
                                  AggLds<ITERS, kFused, K>& S) {
    const int W = A.W, H = A.H;
    const int t = threadIdx.x;
    const int x0 = strip * kStripOut;
    const int c = x0 - 2 * kLMax + t;
    const bool in_img = c >= 0 && c < W;
    const int cc = min(max(c, 0), W - 1);
    const int j = t - kLMax;
    const bool ring_thr = j >= 0 && j < kRingCols;
    // threads without a ring column share two scratch columns
    const int jj = ring_thr ? j : kRingCols + (t & 1);
    const bool out_thr = t >= 2 * kLMax && t < 2 * kLMax + kStripOut && c < W;
    const size_t slice = (size_t)W * H;
    float* out = A.out + (size_t)d * slice;

    if (kFused) {
        for (int i = t; i < 766; i += kStripThreads) S.tabA[i] = A.tabA[i];
        if (t < 65) S.tabC[t] = A.tabC[t];
        if (t <= kLMax) {
            const int L = min(t, A.L1);
            S.ab[t] = A.alpha[L];
            S.ab[kLMax + 1 + t] = A.beta[L];
        }
    }
    if (t < K) S.pbuf[t][0] = 0;  // P(-1) of every prefix row
    // zero column prefixes: rows before the start contribute nothing
    for (int i = t; i < kRing * kRingStride; i += kStripThreads) {
        S.ring1[i] = 0;
        if (ITERS == 2) S.ring2[i] = 0;
    }
    const int cp = A.ref == 0 ? c - d : c + d;
    const int cpc = min(max(cp, 0), W - 1);
    Lane ln;
    ln.rec4 = (uint32_t)(c + A.rec.apron) * 4;
    ln.rec8 = (uint32_t)(c + A.rec.apron) * 8;
    ln.img4 = in_img ? (uint32_t)cc * 4 : kOOB;
    ln.img8 = (uint32_t)cc * 8;
    ln.par4 = (uint32_t)cpc * 4;
    ln.par8 = (uint32_t)cpc * 8;
    ln.col_mask = in_img ? ~0u : 0u;
    ln.par_ok = in_img && cp >= 0 && cp < W ? ~0u : 0u;
    const uint32_t recN = (uint32_t)(A.rec.Wp * (H + 1));
    const uint32_t P4 = (uint32_t)(slice * 4);
    const uint32_t* Iref = A.ref == 0 ? A.rgbL : A.rgbR;
    const uint32_t* Ipar = A.ref == 0 ? A.rgbR : A.rgbL;
    const uint64_t* Cref = A.ref == 0 ? A.cenL : A.cenR;
    const uint64_t* Cpar = A.ref == 0 ? A.cenR : A.cenL;
    AggRes R;
    R.rA = make_rsrc(A.rec.a, recN * 4);
    R.rB = make_rsrc(A.rec.b, recN * 8);
    R.rC = make_rsrc(A.rec.c, recN * 8);
    R.rq = make_rsrc(
        kFused ? (const void*)A.rec.a : (const void*)(A.cost + (size_t)d * slice), P4);
    R.rIr = make_rsrc(kFused ? (const void*)Iref : nullptr, P4);
    R.rIp = make_rsrc(kFused ? (const void*)Ipar : nullptr, P4);
    R.rCr = make_rsrc(kFused ? (const void*)Cref : nullptr, 2 * P4);
    R.rCp = make_rsrc(kFused ? (const void*)Cpar : nullptr, 2 * P4);
    uint32_t* r1 = S.ring1 + jj;
    uint32_t* r2 = S.ring2 + (ITERS == 2 ? jj : 0);
    __syncthreads();

    // warm-up rows so that the first output row sees complete ranges
    const int warm = ITERS == 2 ? 2 * kLMax + 1 : kLMax;
    const int ys = max(0, y0 - warm);
    const int yend = y1 + warm;
    uint32_t cp1 = 0, cp2 = 0;
    uint32_t slot_off = 0;  // ring byte offset of the current row
    RowData<kFused> ra[K], rb[K];
    load_rows<ITERS, kFused, K>(A, ys, ln, R, ra);
    for (int yc = ys; yc < yend; yc += 2 * K) {
        // the next chunk's loads are in flight while this chunk is processed
        load_rows<ITERS, kFused, K>(A, yc + K, ln, R, rb);
        process_rows<ITERS, kFused, K>(yc, y0, y1, W, c, t, ring_thr, out_thr, ln, out, ra, cp1,
                                       cp2, slot_off, r1, r2, S);
        if (yc + K >= yend) break;
        load_rows<ITERS, kFused, K>(A, yc + 2 * K, ln, R, ra);
        process_rows<ITERS, kFused, K>(yc + K, y0, y1, W, c, t, ring_thr, out_thr, ln, out, rb,
                                       cp1, cp2, slot_off, r1, r2, S);
    }
}

// Work item of block b of n, remapped so that the blocks one XCD runs
// (round-robin block -> XCD dispatch) get consecutive items: neighbouring
// strips of the same slice share their apron columns in that XCD's L2.
__device__ inline int xcd_work_item(int b, int n) {
    const int xcd = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

// ===========================================================================
// Winner-take-all (Eq. 3) with parabola sub-pixel refinement; LR check
// ===========================================================================

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
    if (delta_out) {
        float del = 0.f;
        if (subpixel && bd > 0 && bd < D - 1) {
            const float num = m - pl;
            const float den = (m - best) + (pl - best);
            if (den > 0.f) {
                del = num / (2.0f * den);
                del = fminf(fmaxf(del, -0.5f), 0.5f);
            }
        }
        *delta_out = del;
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
