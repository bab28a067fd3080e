// k_aggregate.hip -- aggregation over the adaptive cross region (Eq. 2),
// applied as two stages (horizontal-then-vertical, then
// vertical-then-horizontal), in exact integer arithmetic.
//
// Work decomposition: one workgroup = one disparity slice x one column strip.
// The strip's 256 threads own 256 consecutive columns: 2*kLMax apron columns
// on each side and kStripOut output columns in the middle.  The workgroup
// streams down the image rows, so the vertical apron costs nothing; the
// horizontal apron is re-read from L2.
//
// Per row the four range sums are
//   H1: E1 = row range sum of q             (block prefix scan + 2 LDS reads)
//   V1: S1 = column range sum of E1         (per-column ring of prefix sums)
//       a1 = floor((S1 + N1/2) / N1)        (exact multiply-shift division)
//   V2: E2 = column range sum of a1         (second per-column ring)
//   H2: S2 = row range sum of E2            (block prefix scan + 2 LDS reads)
//       out = RN(S2 / N2) * 2^-20           (reciprocal + one FMA correction)
// Each ring keeps the last kRing column-prefix rows of one column; only the
// thread owning that column touches it, so ring traffic needs no barrier.
// Rows are handled in chunks of kRowChunk so that the two block scans of a
// chunk cost four barriers in total, and the next chunk's loads are issued
// before the current chunk is processed.  The pipeline lags: V1 finalises
// row y - kLMax and H2 row y - 2 kLMax - 1 while H1 consumes row y.
//
// Per-pixel data comes from the packed records written by k_geometry
// (k_census.hip): they carry a zero apron and a zero extra row, so rows and
// columns outside the image read as zeros through buffer loads with a
// per-lane column offset and a uniform row offset (no address arithmetic and
// no bounds branches in the chunk body).  Zero arms and zero division data
// make every range sum of such a row or column zero.
//
// Every sum is an integer (differences of prefix sums taken mod 2^32 are exact
// because every true range sum is below 2^31), so the result does not depend
// on summation order and equals the oracle bit for bit.
//
// The same kernel body also serves the one-call matcher: with kFused the raw
// cost q of Eq. 1 is computed on the fly from the images and census codes
// instead of being read from a cost volume.
#include "dco_internal.h"

namespace {

constexpr int kRingCols = kStripThreads - 2 * kLMax;  // ring columns used: 222
constexpr int kRingStride = 224;
constexpr int kPB = kStripThreads + 4;                // prefix row stride (P[-1] at 0)
constexpr uint32_t kRingBytes = kRing * kRingStride * 4;
constexpr uint32_t kOOB = 0x7fffffffu;                // buffer offset that reads as 0

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
// (pb[k][0] holds 0 from the kernel start).  Two barriers; on return every
// thread sees every row's prefix.
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

// Byte offset inside a ring of the row `back` rows behind the row whose
// slot byte offset is `slot_off` (0 <= back < kRing).  The unsigned minimum
// picks the wrapped value when the subtraction goes below zero.
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

// Work item of block b, remapped so that the blocks one XCD runs (round-robin
// block -> XCD dispatch) get consecutive items: neighbouring strips of the
// same slice share their apron columns in that XCD's L2.
__device__ inline int xcd_work_item(int b, int n) {
    const int xcd = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
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

template <int ITERS, bool kFused>
__device__ inline void load_rows(const AggArgs& A, int yc, const Lane& ln, rsrc_t rA, rsrc_t rB,
                                 rsrc_t rC, rsrc_t rq, rsrc_t rIr, rsrc_t rIp, rsrc_t rCr,
                                 rsrc_t rCp, RowData<kFused> (&rd)[kRowChunk]) {
    const int H = A.H;
    const uint32_t Wp = (uint32_t)A.rec.Wp, W = (uint32_t)A.W;
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k) {
        const int y = yc + k;
        const int y1 = y - kLMax;
        const int yo = ITERS == 2 ? y - 2 * kLMax - 1 : y1;
        // records: rows outside the image map to the zero row H
        const uint32_t ra = (uint32_t)(y < H ? y : H);
        const uint32_t rb = (uint32_t)(y1 >= 0 && y1 < H ? y1 : H);
        const uint32_t rc = (uint32_t)(yo >= 0 && yo < H ? yo : H);
        rd[k].recA = ld32(rA, ln.rec4, ra * Wp * 4);
        rd[k].recB = ld64(rB, ln.rec8, rb * Wp * 8);
        rd[k].recC = ld64(rC, ln.rec8, rc * Wp * 8);
        const uint32_t yq = (uint32_t)min(y, H - 1);
        const uint32_t row_mask = y < H ? ~0u : 0u;
        if (kFused) {
            rd[k].rrgb = ld32(rIr, ln.img4, yq * W * 4);
            rd[k].prgb = ld32(rIp, ln.par4, yq * W * 4);
            rd[k].rcen = ld64(rCr, ln.img8, yq * W * 8);
            rd[k].pcen = ld64(rCp, ln.par8, yq * W * 8);
            rd[k].q = row_mask;
        } else {
            const float v = __builtin_bit_cast(float, ld32(rq, ln.img4, yq * W * 4));
            rd[k].q = (uint32_t)(v * 1048576.0f) & row_mask;
        }
    }
}

template <int ITERS, bool kFused>
__device__ inline void process_rows(int yc, int H, int W, int c, int t, bool ring_thr,
                                    bool out_thr, const Lane& ln, float* __restrict__ out,
                                    RowData<kFused> (&rd)[kRowChunk], uint32_t& cp1,
                                    uint32_t& cp2, uint32_t& slot_off, uint32_t* ring1,
                                    uint32_t* ring2, uint32_t (*pbuf)[kPB],
                                    uint32_t (*wsum)[kRowChunk][4], const float* s_tabA,
                                    const float* s_tabC, const float* s_ab) {
    uint32_t v[kRowChunk];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k) {
        if (kFused) {
            const uint32_t a = rd[k].recA;
            const int lmin = min(min((int)(a & 0xff), (int)((a >> 8) & 0xff)),
                                 min((int)((a >> 16) & 0xff), (int)(a >> 24)));
            const uint32_t s = __builtin_amdgcn_sad_u8(rd[k].rrgb, rd[k].prgb, 0u);
            const int h = __popc(rd[k].rcen.x ^ rd[k].pcen.x) + __popc(rd[k].rcen.y ^ rd[k].pcen.y);
            const float qa = __builtin_rintf(s_ab[lmin] * s_tabA[s]);
            const float qc = __builtin_rintf(s_ab[kLMax + 1 + lmin] * s_tabC[h]);
            const uint32_t qv = ln.par_ok ? (uint32_t)qa + (uint32_t)qc : (1u << 20);
            v[k] = qv & rd[k].q & ln.col_mask;
        } else {
            v[k] = rd[k].q;
        }
    }
    block_scan_rows<kRowChunk>(v, pbuf, wsum[0]);

    uint32_t e2[kRowChunk];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k) {
        // H1: E1 of row y = yc + k, pushed as the column prefix of row y
        {
            const uint32_t a = rd[k].recA;
            const int l = a & 0xff, r = (a >> 8) & 0xff;
            const uint32_t e1 = pbuf[k][t + r + 1] - pbuf[k][t - l];
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
        {   // V1: S1 of row y1 = y - kLMax (prefix rows y1 - u - 1 .. y1 + dn)
            const uint32_t g = rd[k].recB.y;
            const int u = (g >> 16) & 31, dn = (g >> 21) & 31;
            const uint32_t s1 = lds_ld(ring1, ring_off(slot_off, kLMax - dn)) -
                                lds_ld(ring1, ring_off(slot_off, kLMax + u + 1));
            if (ITERS == 2) {
                const uint64_t n = (uint64_t)(s1 + (g & 1023));
                cp2 += (uint32_t)((n * rd[k].recB.x) >> ((g >> 10) & 63));
                lds_st(ring2, ring_off(slot_off, kLMax), cp2);
            } else {
                const int y1 = yc + k - kLMax;
                const uint32_t gc = rd[k].recC.y;
                const float a1 =
                    div_rn(s1, (float)(gc >> 20), __builtin_bit_cast(float, rd[k].recC.x));
                if (out_thr && y1 >= 0 && y1 < H) out[(size_t)y1 * W + c] = a1 * 0x1p-20f;
            }
        }
        slot_off = slot_off + kRingStride * 4 == kRingBytes ? 0u : slot_off + kRingStride * 4;
    }
    if (ITERS == 2) {
        block_scan_rows<kRowChunk>(e2, pbuf, wsum[1]);
        float a2[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {  // H2: S2 of row y - 2 kLMax - 1
            const uint32_t g = rd[k].recC.y;
            const int l = g & 31, r = (g >> 5) & 31;
            const uint32_t s2 = pbuf[k][t + r + 1] - pbuf[k][t - l];
            a2[k] = div_rn(s2, (float)(g >> 20), __builtin_bit_cast(float, rd[k].recC.x)) *
                    0x1p-20f;
        }
        if (out_thr) {
#pragma unroll
            for (int k = 0; k < kRowChunk; ++k) {
                const int y2 = yc + k - 2 * kLMax - 1;
                if (y2 >= 0 && y2 < H) out[(size_t)y2 * W + c] = a2[k];
            }
        }
    }
}

template <int ITERS, bool kFused>
__global__ __launch_bounds__(kStripThreads, 2) void k_agg_stream(AggArgs A) {
    __shared__ uint32_t ring1[kRing * kRingStride];
    __shared__ uint32_t ring2[ITERS == 2 ? kRing * kRingStride : 1];
    __shared__ uint32_t pbuf[kRowChunk][kPB];
    __shared__ __attribute__((aligned(16))) uint32_t wsum[2][kRowChunk][4];
    __shared__ float s_tabA[kFused ? 768 : 1];
    __shared__ float s_tabC[kFused ? 65 : 1];
    __shared__ float s_ab[kFused ? 2 * (kLMax + 1) : 1];

    const int W = A.W, H = A.H;
    const int t = threadIdx.x;
    const int work = xcd_work_item(blockIdx.x, A.nstrips * A.D);
    const int d = work / A.nstrips, strip = work - d * A.nstrips;
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
        for (int i = t; i < 766; i += kStripThreads) s_tabA[i] = A.tabA[i];
        if (t < 65) s_tabC[t] = A.tabC[t];
        if (t <= kLMax) {
            const int L = min(t, A.L1);
            s_ab[t] = A.alpha[L];
            s_ab[kLMax + 1 + t] = A.beta[L];
        }
    }
    if (t < kRowChunk) pbuf[t][0] = 0;  // P(-1) of every prefix row
    // zero column prefixes: rows before the image contribute nothing
    for (int i = t; i < kRing * kRingStride; i += kStripThreads) {
        ring1[i] = 0;
        if (ITERS == 2) ring2[i] = 0;
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
    const rsrc_t rA = make_rsrc(A.rec.a, recN * 4);
    const rsrc_t rB = make_rsrc(A.rec.b, recN * 8);
    const rsrc_t rC = make_rsrc(A.rec.c, recN * 8);
    const uint32_t P4 = (uint32_t)(slice * 4);
    const rsrc_t rq = make_rsrc(
        kFused ? (const void*)A.rec.a : (const void*)(A.cost + (size_t)d * slice), P4);
    const uint32_t* Iref = A.ref == 0 ? A.rgbL : A.rgbR;
    const uint32_t* Ipar = A.ref == 0 ? A.rgbR : A.rgbL;
    const uint64_t* Cref = A.ref == 0 ? A.cenL : A.cenR;
    const uint64_t* Cpar = A.ref == 0 ? A.cenR : A.cenL;
    const rsrc_t rIr = make_rsrc(kFused ? (const void*)Iref : nullptr, P4);
    const rsrc_t rIp = make_rsrc(kFused ? (const void*)Ipar : nullptr, P4);
    const rsrc_t rCr = make_rsrc(kFused ? (const void*)Cref : nullptr, 2 * P4);
    const rsrc_t rCp = make_rsrc(kFused ? (const void*)Cpar : nullptr, 2 * P4);
    uint32_t* r1 = ring1 + jj;
    uint32_t* r2 = ring2 + (ITERS == 2 ? jj : 0);
    __syncthreads();

    uint32_t cp1 = 0, cp2 = 0;
    uint32_t slot_off = 0;  // ring byte offset of row y
    const int nsteps = ITERS == 2 ? H + 2 * kLMax + 1 : H + kLMax;
    RowData<kFused> ra[kRowChunk], rb[kRowChunk];
    load_rows<ITERS, kFused>(A, 0, ln, rA, rB, rC, rq, rIr, rIp, rCr, rCp, ra);
    for (int yc = 0; yc < nsteps; yc += 2 * kRowChunk) {
        // the next chunk's loads are in flight while this chunk is processed
        load_rows<ITERS, kFused>(A, yc + kRowChunk, ln, rA, rB, rC, rq, rIr, rIp, rCr, rCp, rb);
        process_rows<ITERS, kFused>(yc, H, W, c, t, ring_thr, out_thr, ln, out, ra, cp1, cp2,
                                    slot_off, r1, r2, pbuf, wsum, s_tabA, s_tabC, s_ab);
        if (yc + kRowChunk >= nsteps) break;
        load_rows<ITERS, kFused>(A, yc + 2 * kRowChunk, ln, rA, rB, rC, rq, rIr, rIp, rCr, rCp,
                                 ra);
        process_rows<ITERS, kFused>(yc + kRowChunk, H, W, c, t, ring_thr, out_thr, ln, out, rb,
                                    cp1, cp2, slot_off, r1, r2, pbuf, wsum, s_tabA, s_tabC, s_ab);
    }
}

template <int ITERS, bool kFused>
hipError_t launch_stream(const AggArgs& a, hipStream_t st) {
    const int nblk = a.nstrips * a.D;
    hipLaunchKernelGGL((k_agg_stream<ITERS, kFused>), dim3(nblk), dim3(kStripThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aggregate(const float* cost, const AggRecords& rec, int W, int H, int D,
                            int iters, float* out, hipStream_t st) {
    AggArgs a{};
    a.cost = cost;
    a.rec = rec;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, false>(a, st) : launch_stream<2, false>(a, st);
}

hipError_t launch_cost_aggregate(int ref, const uint32_t* rgbL, const uint32_t* rgbR,
                                 const uint64_t* cenL, const uint64_t* cenR,
                                 const AggRecords& rec, int W, int H, int D, int iters,
                                 const float* tabA, const float* tabC, const float* alpha,
                                 const float* beta, int L1, float* out, hipStream_t st) {
    AggArgs a{};
    a.rgbL = rgbL;
    a.rgbR = rgbR;
    a.cenL = cenL;
    a.cenR = cenR;
    a.tabA = tabA;
    a.tabC = tabC;
    a.alpha = alpha;
    a.beta = beta;
    a.rec = rec;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.ref = ref;
    a.L1 = L1;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, true>(a, st) : launch_stream<2, true>(a, st);
}
