// k_contour.hip -- depth contour extraction given the two optical flow
// fields (Sec. 5): gradient amplitude of each flow (Eq. 6-8), bidirectional
// fusion (Eq. 9-12), box filter and normalisation (Sec. 5.2), and Canny on
// the grey image with the depth gate (Sec. 5.3).
//
// Every floating-point value that decides a pixel (the fusion choice, the
// gate) is formed with the same IEEE operations, in the same order, as the
// definition; square roots are correctly rounded (sqrt_rn), so the maps are
// exact functions of the inputs.  The Sobel gradients are exact integers.
// Hysteresis grows strong pixels into 8-connected weak ones: each launch
// iterates inside 64 x 16 tiles in LDS until nothing changes, from one state
// buffer into the other, and the host repeats launches until a launch
// changes nothing.  The fixed point is the set of weak pixels connected to a
// strong one, whatever the order of the growth.
#include "dco_device.h"

namespace {

// Correctly rounded single-precision square root: the hardware root is
// within one ulp, and the exact double squares of the two half-ulp
// boundaries around it pick the rounded value (a float's square root is
// never exactly at a boundary).
__device__ inline float sqrt_rn(float x) {
    if (!(x > 0.0f)) return x == 0.0f ? 0.0f : __builtin_nanf("");
    float y = __builtin_sqrtf(x);
    const double xd = x;
    const float up = __uint_as_float(__float_as_uint(y) + 1u);  // y > 0: the next floats
    const float dn = __uint_as_float(__float_as_uint(y) - 1u);
    const double hi = ((double)y + (double)up) * 0.5, lo = ((double)y + (double)dn) * 0.5;
    if (hi * hi < xd) y = up;
    else if (lo * lo > xd) y = dn;
    return y;
}

__device__ inline float flow_r(const float2* F, int i) {
    const float2 f = F[i];
    return sqrt_rn(f.x * f.x + f.y * f.y);
}

// Eq. 6-8: max(|r(p_right) - r(p)|, |r(p_bottom) - r(p)|), 0 for a missing neighbour.
__device__ inline float flow_amp(const float2* F, int w, int h, int x, int y) {
    const int i = y * w + x;
    const float r = flow_r(F, i);
    const float gu = x + 1 < w ? fabsf(flow_r(F, i + 1) - r) : 0.0f;
    const float gv = y + 1 < h ? fabsf(flow_r(F, i + w) - r) : 0.0f;
    return gu > gv ? gu : gv;
}

// Eq. 9-11: f1 - f0, the flow at p +- rint(e) projected on e = I(p) / |I(p)|.
__device__ inline float flow_score(const float2* F, int w, int h, int x, int y) {
    const int i = y * w + x;
    const float r = flow_r(F, i);
    if (r == 0.0f) return 0.0f;
    const float2 f = F[i];
    const float ex = f.x / r, ey = f.y / r;
    const int sx = (int)rintf(ex), sy = (int)rintf(ey);
    const int x1 = dco::clampi(x + sx, 0, w - 1), y1 = dco::clampi(y + sy, 0, h - 1);
    const int x0 = dco::clampi(x - sx, 0, w - 1), y0 = dco::clampi(y - sy, 0, h - 1);
    const float2 a = F[y1 * w + x1], b = F[y0 * w + x0];
    const float f1 = a.x * ex + a.y * ey;
    const float f0 = b.x * ex + b.y * ey;
    return f1 - f0;
}

// Largest v over the 256-thread block, then one atomic maximum per block
// into one of kContourMaxSlots slots (spread so that thousands of blocks do
// not queue on one address); the maximum does not depend on the order.
template <typename T>
__device__ inline void block_max_to(T v, T* slots) {
    __shared__ T red[4];
    for (int o = 32; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T m = red[0];
        for (int k = 1; k < 4; ++k) m = red[k] > m ? red[k] : m;
        atomicMax(slots + ((blockIdx.x + blockIdx.y * gridDim.x) & (kContourMaxSlots - 1)), m);
    }
}

// The maximum over the slots, for every thread of the block (all threads
// must call it).
template <typename T>
__device__ inline T slots_max(const T* slots) {
    static_assert(kContourMaxSlots == 64, "one slot per lane of the first wavefront");
    __shared__ T m;
    if (threadIdx.x < 64) {
        T v = slots[threadIdx.x];
        for (int o = 32; o > 0; o >>= 1) {
            const T u = __shfl_xor(v, o, 64);
            v = u > v ? u : v;
        }
        if (threadIdx.x == 0) m = v;
    }
    __syncthreads();
    return m;
}

// Eq. 12 per pixel of the flow grid (equal scores keep the larger amplitude).
__global__ __launch_bounds__(256) void k_fuse(const float2* __restrict__ past,
                                              const float2* __restrict__ future, int w, int h,
                                              float* __restrict__ fused) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= w * h) return;
    const int y = i / w, x = i - y * w;
    const float mp = flow_amp(past, w, h, x, y), mf = flow_amp(future, w, h, x, y);
    const float sp = flow_score(past, w, h, x, y), sf = flow_score(future, w, h, x, y);
    fused[i] = sp > sf ? mp : (sf > sp ? mf : (mp > mf ? mp : mf));
}

// Mean over the (2R + 1)^2 window clipped to the grid, summed row by row,
// left to right; the largest mean goes to *mx (non-negative floats order
// like their bit patterns, so an integer maximum is exact).
__global__ __launch_bounds__(256) void k_box(const float* __restrict__ fused, int w, int h, int R,
                                             float* __restrict__ box, unsigned* __restrict__ mx) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    unsigned bits = 0u;  // the bits of a non-negative float order like the float
    if (i < w * h) {
        const int y = i / w, x = i - y * w;
        float s = 0.0f;
        int n = 0;
        for (int yy = max(y - R, 0); yy <= min(y + R, h - 1); ++yy)
            for (int xx = max(x - R, 0); xx <= min(x + R, w - 1); ++xx) {
                s += fused[yy * w + xx];
                ++n;
            }
        const float v = s / (float)n;
        box[i] = v;
        bits = __float_as_uint(v);
    }
    block_max_to(bits, mx);
}

__global__ __launch_bounds__(256) void k_norm(float* __restrict__ box, int n,
                                              const unsigned* __restrict__ mx) {
    const float m = __uint_as_float(slots_max(mx));
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    box[i] = m > 0.0f ? box[i] / m : 0.0f;
}

// Sobel of the census grey (replicated borders): gx, gy and G2 = gx^2 + gy^2
// (exact integers); the largest G2 goes to *mx.  One block per 64 x 4 tile:
// the grey of the tile and a one-pixel ring is computed once into LDS (the
// ring clamped to the image, which replicates the borders), then each
// thread reads its 3 x 3 neighbourhood from there.
constexpr int kSobTW = 64, kSobTH = 4;
__global__ __launch_bounds__(256) void k_sobel(const uint8_t* __restrict__ rgb, int W, int H,
                                               short2* __restrict__ g, int* __restrict__ G2,
                                               int* __restrict__ mx) {
    constexpr int RW = kSobTW + 2, RH = kSobTH + 2, N = RW * RH;
    __shared__ int Yt[RH][RW];
    const int x0 = blockIdx.x * kSobTW, y0 = blockIdx.y * kSobTH, t = threadIdx.x;
    for (int k = t; k < N; k += 256) {
        const int ry = k / RW, rx = k - ry * RW;
        const int xx = dco::clampi(x0 + rx - 1, 0, W - 1), yy = dco::clampi(y0 + ry - 1, 0, H - 1);
        const size_t q = 3 * ((size_t)yy * W + xx);
        Yt[ry][rx] = (int)dco::grey_of((uint32_t)rgb[q] | (uint32_t)rgb[q + 1] << 8 |
                                       (uint32_t)rgb[q + 2] << 16);
    }
    __syncthreads();
    const int tx = t & (kSobTW - 1), ty = t / kSobTW;
    const int x = x0 + tx, y = y0 + ty;
    int v = 0;
    if (x < W && y < H) {
        // Yt[ty + 1 + dy][tx + 1 + dx] is the grey at (x + dx, y + dy), clamped
        const int a = Yt[ty][tx + 2] + 2 * Yt[ty + 1][tx + 2] + Yt[ty + 2][tx + 2] - Yt[ty][tx] -
                      2 * Yt[ty + 1][tx] - Yt[ty + 2][tx];
        const int b = Yt[ty + 2][tx] + 2 * Yt[ty + 2][tx + 1] + Yt[ty + 2][tx + 2] - Yt[ty][tx] -
                      2 * Yt[ty][tx + 1] - Yt[ty][tx + 2];
        const size_t i = (size_t)y * W + x;
        g[i] = make_short2((short)a, (short)b);
        v = a * a + b * b;
        G2[i] = v;
    }
    block_max_to(v, mx);
}

// Suppression along the gradient's sector, the depth gate on the flow grid,
// and the double threshold: state 2 strong, 1 weak, 0 none.  MI = the
// normalised magnitude sqrt(G2 / max G2).
__global__ __launch_bounds__(256) void k_nms(const short2* __restrict__ g,
                                             const int* __restrict__ G2, int W, int H,
                                             const float* __restrict__ Mn, int w, int h,
                                             const int* __restrict__ mxp, float Thigh, float Tlow,
                                             float Tdepth, uint8_t* __restrict__ st,
                                             float* __restrict__ MI) {
    const int mx = slots_max(mxp);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= W * H) return;
    const int y = i / W, x = i - y * W;
    const int v = G2[i];
    if (MI) MI[i] = mx > 0 ? sqrt_rn((float)((double)v / (double)mx)) : 0.0f;
    const short2 gi = g[i];
    const int ax = abs((int)gi.x), ay = abs((int)gi.y);
    int dx, dy;
    if (128 * ay < 53 * ax) {
        dx = 1;
        dy = 0;
    } else if (128 * ax < 53 * ay) {
        dx = 0;
        dy = 1;
    } else if ((gi.x > 0) == (gi.y > 0)) {
        dx = 1;
        dy = 1;
    } else {
        dx = 1;
        dy = -1;
    }
    const int xa = x - dx, ya = y - dy, xb = x + dx, yb = y + dy;
    const int ga = xa >= 0 && xa < W && ya >= 0 && ya < H ? G2[ya * W + xa] : 0;
    const int gb = xb >= 0 && xb < W && yb >= 0 && yb < H ? G2[yb * W + xb] : 0;
    uint8_t s = 0;
    if (v > ga && v >= gb) {
        const float gate = Mn[min(y / 2, h - 1) * w + min(x / 2, w - 1)];
        if (!(gate < Tdepth)) {
            const double th = (double)Thigh * (double)Thigh * (double)mx;
            const double tl = (double)Tlow * (double)Tlow * (double)mx;
            const double dv = (double)v;
            s = dv > th ? 2 : (dv > tl ? 1 : 0);
        }
    }
    st[i] = s;
}

// One hysteresis launch: tile + 1-pixel halo from `in` to LDS, grow strong
// pixels into 8-neighbouring weak ones inside the tile until it is stable,
// write the tile to `out`; *changed is set if any pixel changed.
constexpr int kHTW = 64, kHTH = 16;

__global__ __launch_bounds__(256) void k_hyst(const uint8_t* __restrict__ in, int W, int H,
                                              uint8_t* __restrict__ out,
                                              const int* __restrict__ prev,
                                              int* __restrict__ changed) {
    __shared__ uint8_t T[kHTH + 2][kHTW + 2];
    // the previous launch of the group changed nothing: the state is final
    // (the same value for every thread of every block)
    if (prev && *prev == 0) return;
    const int x0 = blockIdx.x * kHTW, y0 = blockIdx.y * kHTH;
    for (int k = threadIdx.x; k < (kHTH + 2) * (kHTW + 2); k += 256) {
        const int ty = k / (kHTW + 2), tx = k - ty * (kHTW + 2);
        const int x = x0 + tx - 1, y = y0 + ty - 1;
        T[ty][tx] = x >= 0 && x < W && y >= 0 && y < H ? in[(size_t)y * W + x] : 0;
    }
    __syncthreads();
    bool any = false;
    for (;;) {
        bool grew = false;
        for (int k = threadIdx.x; k < kHTH * kHTW; k += 256) {
            const int ty = k / kHTW + 1, tx = k % kHTW + 1;
            if (T[ty][tx] != 1) continue;
            const bool hit = T[ty - 1][tx - 1] == 2 || T[ty - 1][tx] == 2 ||
                             T[ty - 1][tx + 1] == 2 || T[ty][tx - 1] == 2 ||
                             T[ty][tx + 1] == 2 || T[ty + 1][tx - 1] == 2 ||
                             T[ty + 1][tx] == 2 || T[ty + 1][tx + 1] == 2;
            if (hit) {
                T[ty][tx] = 2;
                grew = true;
            }
        }
        any = any || grew;
        if (!__syncthreads_or(grew)) break;
    }
    for (int k = threadIdx.x; k < kHTH * kHTW; k += 256) {
        const int ty = k / kHTW, tx = k % kHTW;
        const int x = x0 + tx, y = y0 + ty;
        if (x < W && y < H) out[(size_t)y * W + x] = T[ty + 1][tx + 1];
    }
    if (__syncthreads_or(any) && threadIdx.x == 0) *changed = 1;
}

__global__ __launch_bounds__(256) void k_edges(const uint8_t* __restrict__ st, int n,
                                               uint8_t* __restrict__ B) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) B[i] = st[i] == 2;
}

__global__ void k_zero2(unsigned* a, int* b) {
    if (threadIdx.x < kContourMaxSlots) {
        a[threadIdx.x] = 0u;
        b[threadIdx.x] = 0;
    }
}

__global__ void k_zero1(int* a, int n) {
    if ((int)threadIdx.x < n) a[threadIdx.x] = 0;
}

inline dim3 grid1(int n) { return dim3((n + 255) / 256); }

}  // namespace

hipError_t launch_contour_maps(const float* past, const float* future, int w, int h, int R,
                               const uint8_t* rgb, int W, int H, float Thigh, float Tlow,
                               float Tdepth, const ContourBufs& b, float* Mn, float* MI,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(kContourMaxSlots), 0, st, b.box_max, b.g2_max);
    hipLaunchKernelGGL(k_fuse, grid1(w * h), dim3(256), 0, st,
                       reinterpret_cast<const float2*>(past),
                       reinterpret_cast<const float2*>(future), w, h, b.fused);
    hipLaunchKernelGGL(k_box, grid1(w * h), dim3(256), 0, st, b.fused, w, h, R, Mn, b.box_max);
    hipLaunchKernelGGL(k_norm, grid1(w * h), dim3(256), 0, st, Mn, w * h, b.box_max);
    hipLaunchKernelGGL(k_sobel, dim3((W + kSobTW - 1) / kSobTW, (H + kSobTH - 1) / kSobTH),
                       dim3(256), 0, st, rgb, W, H, b.g, b.G2, b.g2_max);
    hipLaunchKernelGGL(k_nms, grid1(W * H), dim3(256), 0, st, b.g, b.G2, W, H, Mn, w, h, b.g2_max,
                       Thigh, Tlow, Tdepth, b.state[0], MI);
    return hipGetLastError();
}

// Launch k of the group reads state[parity ^ (k & 1)] and writes the other
// buffer; kHystGroup is even, so the group's last output is state[parity].
hipError_t launch_contour_hyst_group(const ContourBufs& b, int W, int H, int parity,
                                     hipStream_t st) {
    static_assert(kHystGroup % 2 == 0 && kHystGroup <= 64, "even group, one flag per lane");
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, st, b.changed, kHystGroup);
    const dim3 grid((W + kHTW - 1) / kHTW, (H + kHTH - 1) / kHTH);
    for (int k = 0; k < kHystGroup; ++k) {
        const int p = parity ^ (k & 1);
        hipLaunchKernelGGL(k_hyst, grid, dim3(256), 0, st, b.state[p], W, H, b.state[1 - p],
                           k ? (const int*)(b.changed + k - 1) : (const int*)nullptr,
                           b.changed + k);
    }
    return hipGetLastError();
}

hipError_t launch_contour_edges(const ContourBufs& b, int W, int H, int parity, uint8_t* B,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_edges, grid1(W * H), dim3(256), 0, st, b.state[parity], W * H, B);
    return hipGetLastError();
}
