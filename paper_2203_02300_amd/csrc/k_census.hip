// k_census.hip -- grey conversion, census codes and cross-support arms of one
// image (paper Sec. 4.1; the C_census term of Eq. 1), and the per-pixel
// division data of the aggregation.
//
// One workgroup of 256 threads covers a 64 x 16 pixel tile.  The tile plus a
// kLMax-pixel apron (edge-clamped) is staged once in LDS as packed RGB words;
// grey levels of the tile plus the census apron go to a second LDS array.
// Every census compare and every arm step then reads LDS only.
#include "dco_internal.h"

namespace {

constexpr int kTW = 64, kTH = 16;
constexpr int kRW = kTW + 2 * kLMax, kRH = kTH + 2 * kLMax;  // staged RGB region
constexpr int kMaxHW = 4, kMaxHH = 4;                          // census half-window limits
constexpr int kGW = kTW + 2 * kMaxHW, kGH = kTH + 2 * kMaxHH;  // staged grey region

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

__global__ __launch_bounds__(256) void k_census_arms(const uint8_t* __restrict__ rgb, int W,
                                                     int H, int cw, int ch, int L1, int tau1,
                                                     uint64_t* __restrict__ census,
                                                     uint32_t* __restrict__ arms,
                                                     uint32_t* __restrict__ rgb_packed) {
    __shared__ uint32_t s_rgb[kRH][kRW];
    __shared__ uint32_t s_grey[kGH][kGW];
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
    const int t = threadIdx.x;

    for (int i = t; i < kRW * kRH; i += 256) {
        int ry = i / kRW, rx = i - ry * kRW;
        int gx = clampi(x0 - kLMax + rx, 0, W - 1), gy = clampi(y0 - kLMax + ry, 0, H - 1);
        const uint8_t* p = rgb + 3 * ((size_t)gy * W + gx);
        s_rgb[ry][rx] = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
    }
    __syncthreads();
    for (int i = t; i < kGW * kGH; i += 256) {
        int gy = i / kGW, gx = i - gy * kGW;
        s_grey[gy][gx] = grey_of(s_rgb[gy + kLMax - kMaxHH][gx + kLMax - kMaxHW]);
    }
    __syncthreads();

    const int hw = cw >> 1, hh = ch >> 1;
    const int tx = t & 63;
    for (int k = 0; k < kTH / 4; ++k) {
        const int ty = (t >> 6) + 4 * k;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H) continue;
        // census: neighbours row-major, centre skipped, strict "darker than centre"
        const uint32_t c = s_grey[ty + kMaxHH][tx + kMaxHW];
        uint64_t code = 0;
        int bit = 0;
        for (int dy = -hh; dy <= hh; ++dy) {
            for (int dx = -hw; dx <= hw; ++dx) {
                if (dy == 0 && dx == 0) continue;
                uint32_t v = s_grey[ty + kMaxHH + dy][tx + kMaxHW + dx];
                code |= (uint64_t)(v < c) << bit;
                ++bit;
            }
        }
        census[(size_t)y * W + x] = code;

        // arms: stop at the border, at L1, or at the first step whose colour
        // differs from the centre by tau1 or more in some channel
        const int rx = tx + kLMax, ry = ty + kLMax;
        const uint32_t cp = s_rgb[ry][rx];
        if (rgb_packed) rgb_packed[(size_t)y * W + x] = cp;
        int al = 0, ar = 0, au = 0, ad = 0;
        const int ml = min(L1, x), mr = min(L1, W - 1 - x);
        const int mu = min(L1, y), md = min(L1, H - 1 - y);
        while (al < ml && close_rgb(s_rgb[ry][rx - al - 1], cp, tau1)) ++al;
        while (ar < mr && close_rgb(s_rgb[ry][rx + ar + 1], cp, tau1)) ++ar;
        while (au < mu && close_rgb(s_rgb[ry - au - 1][rx], cp, tau1)) ++au;
        while (ad < md && close_rgb(s_rgb[ry + ad + 1][rx], cp, tau1)) ++ad;
        arms[(size_t)y * W + x] =
            (uint32_t)al | ((uint32_t)ar << 8) | ((uint32_t)au << 16) | ((uint32_t)ad << 24);
    }
}

// Region pixel counts and the packed aggregation records of every pixel:
//   N1 = sum over y' in [y-u, y+dn] of (l(x,y') + r(x,y') + 1)
//   N2 = sum over x' in [x-l, x+r] of (u(x',y) + dn(x',y) + 1)
// Stage-1 rounding uses sh = 31 + ceil(log2 N1) and m = ceil(2^sh / N1) <
// 2^32, so floor(n / N1) = (n * m) >> sh for every 0 <= n < 2^31 (N1 <= 2^11).
// The final division uses (N, RN(1/N)) with N = N2 (two stages) or N1 (one).
// Record layout: see AggRecords.
__global__ __launch_bounds__(256) void k_geometry(const uint32_t* __restrict__ arms, int W, int H,
                                                  int iters, AggRecords rec) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const uint32_t a = arms[(size_t)y * W + x];
    const uint32_t l = a & 0xff, r = (a >> 8) & 0xff, u = (a >> 16) & 0xff, dn = a >> 24;
    uint32_t n1 = 0, n2 = 0;
    // arms come from k_census_arms and stay inside the image; the clamps only
    // keep a corrupted arms buffer from reading outside it
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

}  // namespace

hipError_t launch_census_arms(const uint8_t* rgb, int W, int H, int cw, int ch, int L1, int tau1,
                              uint64_t* census, uint32_t* arms, uint32_t* rgb_packed,
                              hipStream_t st) {
    dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH);
    hipLaunchKernelGGL(k_census_arms, grid, dim3(256), 0, st, rgb, W, H, cw, ch, L1, tau1, census,
                       arms, rgb_packed);
    return hipGetLastError();
}

hipError_t launch_geometry(const uint32_t* arms, int W, int H, int iters, const AggRecords& rec,
                           hipStream_t st) {
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(k_geometry, grid, dim3(256), 0, st, arms, W, H, iters, rec);
    return hipGetLastError();
}
