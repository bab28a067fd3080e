"""Seeded synthetic rectified stereo pairs (slanted-plane scenes).

The paper's own inputs (INDEMIND indoor frames at 1280x720, stereo run at a
quarter of the area, Sec. 7.1 and Sec. 4; Middlebury 2014 for Fig. 3) are not
available, so seeded synthetic scenes of the same shapes stand in for them.

This module renders scenes only.  It holds none of the matcher's arithmetic
(no grey conversion, census, arms, costs or aggregation), so both the CPU
oracle and the GPU library can be fed from it.

Every generator returns a dict with
  ``left``, ``right``   : ``H x W x 3`` uint8, row-major, channel-interleaved
  ``disp``              : ``H x W`` float32 ground-truth disparity of the left
                          view (right pixel = left pixel shifted by ``-disp``)
  ``occluded``          : ``H x W`` bool, True where the left pixel has no
                          visible counterpart in the right view
  ``W``, ``H``, ``D``   : sizes, ``seed``
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Texture functions
# ---------------------------------------------------------------------------


def _lattice(rng, ny, nx):
    return rng.random((ny + 2, nx + 2))


def _smooth(t):
    return t * t * (3.0 - 2.0 * t)


def _value_noise(lat, period, u, v):
    """Value noise on a lattice of spacing ``period`` evaluated at (u, v)."""
    gu = u / period
    gv = v / period
    iu = np.floor(gu).astype(np.int64)
    iv = np.floor(gv).astype(np.int64)
    fu = _smooth(gu - iu)
    fv = _smooth(gv - iv)
    ny, nx = lat.shape
    iu0 = np.clip(iu, 0, nx - 2)
    iv0 = np.clip(iv, 0, ny - 2)
    a = lat[iv0, iu0]
    b = lat[iv0, iu0 + 1]
    c = lat[iv0 + 1, iu0]
    d = lat[iv0 + 1, iu0 + 1]
    top = a + (b - a) * fu
    bot = c + (d - c) * fu
    return top + (bot - top) * fv


class _Texture:
    """Per-layer colour texture T(u, v) in left-image coordinates.

    T = base_c + amp * ((1 - w) * (fractal - 0.5) + w * (uniform_c - 0.5))
    with a 4-octave fractal value noise (base period 32 px) shared by the
    three channels and a per-channel per-texel uniform component that is
    bilinearly interpolated at fractional positions.
    """

    def __init__(self, rng, W, H, amp, w_uniform, octaves=4, period=32.0):
        self.amp = float(amp)
        self.w = float(w_uniform)
        self.base = rng.uniform(60.0, 195.0, size=3)
        self.octaves = []
        p = float(period)
        for _ in range(octaves):
            ny = int(np.ceil(H / p)) + 2
            nx = int(np.ceil((W + 2) / p)) + 2
            self.octaves.append((p, _lattice(rng, ny, nx)))
            p /= 2.0
        # per-texel uniform component, one extra column for interpolation
        self.unif = rng.random((H, W + 2, 3))

    def __call__(self, u, v):
        """Sample at float column ``u`` and integer row ``v`` (same shapes)."""
        f = np.zeros(u.shape, dtype=np.float64)
        s = 0.0
        amp = 1.0
        for p, lat in self.octaves:
            f += amp * _value_noise(lat, p, u, v.astype(np.float64))
            s += amp
            amp *= 0.5
        f /= s
        Wt = self.unif.shape[1]
        uc = np.clip(u, 0.0, Wt - 1.000001)
        iu = np.floor(uc).astype(np.int64)
        fu = (uc - iu)[..., None]
        vi = v.astype(np.int64)
        un = self.unif[vi, iu] * (1.0 - fu) + self.unif[vi, np.minimum(iu + 1, Wt - 1)] * fu
        val = self.base[None, :] if u.ndim == 1 else self.base
        val = val + self.amp * ((1.0 - self.w) * (f[..., None] - 0.5) + self.w * (un - 0.5))
        return val


# ---------------------------------------------------------------------------
# Config C1: fronto-parallel planes, integer disparities, forward warp
# ---------------------------------------------------------------------------


def make_fronto_pair(W=64, H=48, D=16, seed=1, n_rects=2):
    """Back plane + ``n_rects`` rectangles at integer disparities in [1, D-1].

    Uniform U{0..255} RGB texture.  The right image is the forward warp
    ``R(x - d, y) = L(x, y)`` with a z-buffer (the larger disparity wins);
    holes are filled with fresh uniform texture.  No noise.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    L = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    disp = np.empty((H, W), dtype=np.int64)
    disp[:] = rng.integers(1, max(2, D // 3))
    for _ in range(n_rects):
        rw = int(rng.integers(W // 6, W // 2))
        rh = int(rng.integers(H // 6, H // 2))
        x0 = int(rng.integers(0, W - rw))
        y0 = int(rng.integers(0, H - rh))
        disp[y0:y0 + rh, x0:x0 + rw] = rng.integers(D // 3, D)
    R = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)  # hole fill
    zbuf = np.full((H, W), -1, dtype=np.int64)
    owner = np.full((H, W), -1, dtype=np.int64)
    for y in range(H):
        for x in range(W):
            xr = x - disp[y, x]
            if xr < 0:
                continue
            if disp[y, x] > zbuf[y, xr]:
                zbuf[y, xr] = disp[y, x]
                owner[y, xr] = x
                R[y, xr] = L[y, x]
    occ = np.ones((H, W), dtype=bool)
    for y in range(H):
        for xr in range(W):
            if owner[y, xr] >= 0:
                occ[y, owner[y, xr]] = False
    return dict(left=L, right=R, disp=disp.astype(np.float32), occluded=occ,
                W=W, H=H, D=D, seed=seed)


# ---------------------------------------------------------------------------
# Configs C2 / C3: slanted planes, Perlin + uniform texture, noise
# ---------------------------------------------------------------------------


def _plane_layers(rng, W, H, D, n_planes, n_boxes, dmin, dmax, box_range):
    cx, cy = W / 2.0, H / 2.0
    layers = []
    for i in range(n_planes):
        for _ in range(200):
            a = rng.uniform(dmin, dmax)
            b = rng.uniform(-0.04, 0.04)
            c = rng.uniform(-0.04, 0.04) * (D / 64.0)
            if i == 0:
                rect = (0, 0, W, H)
            else:
                rw = int(rng.integers(W // 8, W // 2))
                rh = int(rng.integers(H // 8, H // 2))
                x0 = int(rng.integers(0, W - rw))
                y0 = int(rng.integers(0, H - rh))
                rect = (x0, y0, x0 + rw, y0 + rh)
            xs = np.array([rect[0], rect[2] - 1], dtype=np.float64)
            ys = np.array([rect[1], rect[3] - 1], dtype=np.float64)
            corners = a + b * (xs[:, None] - cx) + c * (ys[None, :] - cy)
            if corners.min() >= dmin and corners.max() <= dmax:
                break
        layers.append(dict(a=a, b=b, c=c, rect=rect))
    for _ in range(n_boxes):
        a = rng.uniform(*box_range)
        rw = int(rng.integers(W // 10, W // 4))
        rh = int(rng.integers(H // 10, H // 3))
        x0 = int(rng.integers(0, W - rw))
        y0 = int(rng.integers(0, H - rh))
        layers.append(dict(a=a, b=0.0, c=0.0, rect=(x0, y0, x0 + rw, y0 + rh)))
    # back to front: larger mean disparity is nearer and drawn later
    def mean_d(l):
        x0, y0, x1, y1 = l["rect"]
        return l["a"] + l["b"] * ((x0 + x1 - 1) / 2.0 - cx) + l["c"] * ((y0 + y1 - 1) / 2.0 - cy)
    bg = layers[0]
    rest = sorted(layers[1:], key=mean_d)
    return [bg] + rest, cx, cy


def _texture_for(rng, W, H):
    kind = rng.integers(0, 3)
    if kind == 0:      # dense texture: short arms
        amp, w = rng.uniform(150, 230), 0.5
    elif kind == 1:    # medium
        amp, w = rng.uniform(80, 160), 0.1
    else:              # weak texture: long arms
        amp, w = rng.uniform(30, 60), 0.03
    return _Texture(rng, W, H, amp, w)


def make_slanted_pair(W=640, H=480, D=64, seed=2, n_planes=6, n_boxes=0,
                      dmin=4.0, dmax=None, box_range=None, noise_sigma=2.0,
                      gain_range=None, occl_strip_frac=0.0):
    """Slanted planes ``d = a + b (x - cx) + c (y - cy)`` drawn back to front.

    The left view samples each layer's texture at integer pixels; the right
    view is rendered by inverse mapping ``x_l = (x_r + a - b cx + c (y - cy)) /
    (1 - b)`` with bilinear sampling of the per-texel component.  Optional right
    gain (one scalar per pair, applied before noise), Gaussian noise of
    ``noise_sigma`` on both views, then rounding and clipping to uint8.
    Optional vertical strips of fresh texture in the right view (3 % of the
    columns in strips 4..16 px wide) are marked occluded in the ground truth.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if dmax is None:
        dmax = float(D - 4)
    if box_range is None:
        box_range = (0.78 * D, 0.97 * D)
    layers, cx, cy = _plane_layers(rng, W, H, D, n_planes, n_boxes, dmin, dmax, box_range)
    texs = [_texture_for(rng, W, H) for _ in layers]
    if gain_range is not None:
        gain = rng.uniform(*gain_range)
    else:
        gain = 1.0

    ys, xs = np.mgrid[0:H, 0:W]
    xs = xs.astype(np.float64)
    Lf = np.zeros((H, W, 3))
    Rf = np.zeros((H, W, 3))
    labL = np.full((H, W), -1, dtype=np.int64)
    labR = np.full((H, W), -1, dtype=np.int64)
    dispL = np.zeros((H, W))
    for k, (ly, tex) in enumerate(zip(layers, texs)):
        x0, y0, x1, y1 = ly["rect"]
        m = (xs >= x0) & (xs < x1) & (ys >= y0) & (ys < y1)
        if m.any():
            Lf[m] = tex(xs[m], ys[m])
            labL[m] = k
            dispL[m] = ly["a"] + ly["b"] * (xs[m] - cx) + ly["c"] * (ys[m] - cy)
        # right view: inverse map every right pixel into this layer
        xl = (xs + ly["a"] - ly["b"] * cx + ly["c"] * (ys - cy)) / (1.0 - ly["b"])
        mr = (xl >= x0) & (xl <= x1 - 1) & (ys >= y0) & (ys < y1)
        if mr.any():
            Rf[mr] = tex(xl[mr], ys[mr])
            labR[mr] = k

    # occlusion: the left pixel's own layer must be the visible one at x - d
    xr = xs - dispL
    occ = xr < 0
    vis = np.full((H, W), -1, dtype=np.int64)
    xr_c = np.clip(xr, 0, W - 1)
    for k, ly in enumerate(layers):
        x0, y0, x1, y1 = ly["rect"]
        xl = (xr_c + ly["a"] - ly["b"] * cx + ly["c"] * (ys - cy)) / (1.0 - ly["b"])
        hit = (xl >= x0) & (xl <= x1 - 1) & (ys >= y0) & (ys < y1)
        vis[hit] = k
    occ |= vis != labL

    if occl_strip_frac > 0:
        ncols = int(round(occl_strip_frac * W))
        covered = 0
        strip = np.zeros(W, dtype=bool)
        while covered < ncols:
            sw = int(rng.integers(4, 17))
            sx = int(rng.integers(0, W - sw))
            strip[sx:sx + sw] = True
            covered = int(strip.sum())
        fresh = rng.integers(0, 256, size=(H, int(strip.sum()), 3)).astype(np.float64)
        Rf[:, strip] = fresh
        xri = np.clip(np.rint(xr).astype(np.int64), 0, W - 1)
        occ |= strip[xri]

    Rf = Rf * gain
    if noise_sigma > 0:
        Lf = Lf + rng.normal(0.0, noise_sigma, size=Lf.shape)
        Rf = Rf + rng.normal(0.0, noise_sigma, size=Rf.shape)
    L = np.clip(np.rint(Lf), 0, 255).astype(np.uint8)
    R = np.clip(np.rint(Rf), 0, 255).astype(np.uint8)
    return dict(left=L, right=R, disp=dispL.astype(np.float32), occluded=occ,
                W=W, H=H, D=D, seed=seed)


# ---------------------------------------------------------------------------
# Small structured inputs for invariants
# ---------------------------------------------------------------------------


def make_shift_pair(W, H, d0, seed, texture="uniform"):
    """Right view = left view shifted left by ``d0`` columns.

    ``R(x, y) = L(x + d0, y)``; the rightmost ``d0`` columns of R are fresh.
    ``texture`` is ``"uniform"`` (U{0..255} per channel) or ``"patches"``
    (uniform texture overlaid with constant rectangles, so arms grow long).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    L = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    if texture == "patches":
        for _ in range(max(2, (W * H) // 600)):
            rw = int(rng.integers(4, max(5, W // 3)))
            rh = int(rng.integers(4, max(5, H // 3)))
            x0 = int(rng.integers(0, max(1, W - rw)))
            y0 = int(rng.integers(0, max(1, H - rh)))
            L[y0:y0 + rh, x0:x0 + rw] = rng.integers(0, 256, size=3, dtype=np.uint8)
    R = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    if d0 > 0:
        R[:, :W - d0] = L[:, d0:]
    else:
        R[:] = L
    disp = np.full((H, W), float(d0), dtype=np.float32)
    occ = np.zeros((H, W), dtype=bool)
    occ[:, :d0] = True
    return dict(left=L, right=R, disp=disp, occluded=occ, W=W, H=H, D=None, seed=seed)


def make_patchwork(W, H, seed, n=None, noise=0):
    """Piecewise-constant colour rectangles (optionally with small noise)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    img = np.empty((H, W, 3), dtype=np.int64)
    img[:] = rng.integers(0, 256, size=3)
    if n is None:
        n = max(3, (W * H) // 300)
    for _ in range(n):
        rw = int(rng.integers(2, max(3, W // 2)))
        rh = int(rng.integers(2, max(3, H // 2)))
        x0 = int(rng.integers(0, max(1, W - rw)))
        y0 = int(rng.integers(0, max(1, H - rh)))
        img[y0:y0 + rh, x0:x0 + rw] = rng.integers(0, 256, size=3)
    if noise:
        img = img + rng.integers(-noise, noise + 1, size=img.shape)
    return np.clip(img, 0, 255).astype(np.uint8)


# ---------------------------------------------------------------------------
# The five workload configurations
# ---------------------------------------------------------------------------

BATCH_SIZES = ((320, 240), (640, 480), (960, 540), (1280, 720))
BATCH_DISPS = (32, 64, 96, 128)


def config_c1(seed=1):
    """64x48, D=16: three fronto-parallel planes, uniform texture."""
    return make_fronto_pair(64, 48, 16, seed)


def config_c2(seed=2):
    """640x480, D=64: 6 slanted planes (d in 4..60), noise 2, 3 % occluded strips."""
    return make_slanted_pair(640, 480, 64, seed, n_planes=6, dmin=4.0, dmax=60.0,
                             noise_sigma=2.0, occl_strip_frac=0.03)


def config_c3(seed=3):
    """1280x720, D=128: 10 slanted planes + 2 boxes, noise 2, right gain 0.9..1.1."""
    return make_slanted_pair(1280, 720, 128, seed, n_planes=10, n_boxes=2, dmin=4.0,
                             dmax=120.0, box_range=(100.0, 124.0), noise_sigma=2.0,
                             gain_range=(0.9, 1.1))


def batch_shapes(n=32, seed0=100):
    """Shapes (W, H, D) of the batched workload, one per seed."""
    out = []
    for i in range(n):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        W, H = BATCH_SIZES[int(rng.integers(0, 4))]
        D = BATCH_DISPS[int(rng.integers(0, 4))]
        out.append((W, H, D))
    return out


def config_c4(n=32, seed0=100):
    """Batched: ``n`` pairs of mixed sizes and disparity ranges."""
    pairs = []
    for i, (W, H, D) in enumerate(batch_shapes(n, seed0)):
        seed = seed0 + i
        if W <= 640:
            p = make_slanted_pair(W, H, D, seed, n_planes=6, dmin=4.0, dmax=D - 4.0,
                                  noise_sigma=2.0, occl_strip_frac=0.03)
        else:
            p = make_slanted_pair(W, H, D, seed, n_planes=10, n_boxes=2, dmin=4.0,
                                  dmax=D - 8.0, box_range=(0.8 * D, 0.97 * D),
                                  noise_sigma=2.0, gain_range=(0.9, 1.1))
        pairs.append(p)
    return pairs


def config_c5(n=8, seed0=200, W=640, H=480, D=64):
    """Differentiable: ``n`` C2-style pairs."""
    return [make_slanted_pair(W, H, D, seed0 + i, n_planes=6, dmin=4.0, dmax=D - 4.0,
                              noise_sigma=2.0, occl_strip_frac=0.03) for i in range(n)]


def densify_inputs(W=640, H=360, seed=7, fB=1000.0, keep=0.7):
    """Inputs of the depth densification (Eq. 13-20) from a slanted-plane
    scene's ground truth: the sparse depth ``Ds`` (fB / disparity on a random
    ``keep`` fraction of the pixels, 0 elsewhere), the previous frame's depth
    ``Dpre`` (the ground truth scaled by 1 + N(0, 0.01) on half of the pixels,
    0 elsewhere), the binary depth contour ``Bdp`` (pixels with a 4-neighbour
    whose ground-truth disparity differs by more than 1), and the two maps
    ``Mfuse`` and ``MI`` in [0, 1] (smooth value noise standing in for the
    outputs of Sec. 5, which are not built here).  All H x W float32 except
    ``Bdp`` (uint8)."""
    scene = make_slanted_pair(W, H, 64, seed, n_planes=6, n_boxes=2, dmin=4.0, dmax=60.0,
                              noise_sigma=0.0)
    rng = np.random.default_rng(seed + 1000)
    disp = scene["disp"].astype(np.float64)
    depth = fB / np.maximum(disp, 1e-3)
    Ds = np.where(rng.random((H, W)) < keep, depth, 0.0)
    Dpre = np.where(rng.random((H, W)) < 0.5, depth * (1.0 + 0.01 * rng.normal(size=(H, W))), 0.0)
    jump = np.zeros((H, W), bool)
    dx = np.abs(np.diff(disp, axis=1)) > 1.0
    dy = np.abs(np.diff(disp, axis=0)) > 1.0
    jump[:, :-1] |= dx
    jump[:, 1:] |= dx
    jump[:-1, :] |= dy
    jump[1:, :] |= dy
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    lat1, lat2 = _lattice(rng, H // 16 + 2, W // 16 + 2), _lattice(rng, H // 16 + 2, W // 16 + 2)
    Mfuse = _value_noise(lat1, 16.0, xs, ys)
    MI = _value_noise(lat2, 16.0, xs, ys)
    return dict(Ds=Ds.astype(np.float32), Dpre=Dpre.astype(np.float32),
                Bdp=jump.astype(np.uint8), Mfuse=np.clip(Mfuse, 0, 1).astype(np.float32),
                MI=np.clip(MI, 0, 1).astype(np.float32), depth=depth.astype(np.float32),
                W=W, H=H, seed=seed)


def contour_inputs(W=1280, H=720, seed=11):
    """Inputs of the depth contour filter (Sec. 5): the middle colour frame
    (a slanted-plane scene's left view, W x H x 3 uint8) and the past and
    future optical flows on the quarter grid (H/2 x W/2 x 2 float32): the
    foreground boxes of the scene move by +v towards the future frame and by
    -v towards the past one, with the motion spread over a few pixels at the
    box borders and N(0, 0.002) noise, while the background stays still."""
    scene = make_slanted_pair(W, H, 64, seed, n_planes=4, n_boxes=3, dmin=4.0, dmax=40.0,
                              noise_sigma=2.0)
    rng = np.random.default_rng(seed + 2000)
    h, w = H // 2, W // 2
    disp = scene["disp"][: 2 * h : 2, : 2 * w : 2].astype(np.float64)
    fg = disp > np.percentile(disp, 80)  # the nearest surfaces move
    m = fg.astype(np.float64)
    for _ in range(3):  # spread the motion over the borders
        m = (m + np.roll(m, 1, 0) + np.roll(m, -1, 0) + np.roll(m, 1, 1) + np.roll(m, -1, 1)) / 5
    v = rng.uniform(1.0, 4.0, 2)
    fut = np.stack([m * v[0], m * v[1]], -1) + rng.normal(0, 0.002, (h, w, 2))
    past = np.stack([-m * v[0], -m * v[1]], -1) + rng.normal(0, 0.002, (h, w, 2))
    return dict(rgb=scene["left"], past=past.astype(np.float32), future=fut.astype(np.float32),
                W=W, H=H, seed=seed)
