"""Independent numpy formulations used to pin the oracle (tests only).

These are written differently from the oracle on purpose: vectorised shifts
instead of per-pixel loops, explicit pixel-set enumeration instead of
separable sums, and real-valued (float64) arithmetic for the shadow of
Eq. 1 and Eq. 2.  They are slow and meant for tiny images.
"""
from __future__ import annotations

import math

import numpy as np


def census_shift(Y, cw=9, ch=7):
    """Census by comparing the edge-padded image with shifted copies."""
    Y = Y.astype(np.int64)
    H, W = Y.shape
    hw, hh = cw // 2, ch // 2
    pad = np.pad(Y, ((hh, hh), (hw, hw)), mode="edge")
    code = np.zeros((H, W), dtype=np.uint64)
    k = 0
    for dy in range(-hh, hh + 1):
        for dx in range(-hw, hw + 1):
            if dy == 0 and dx == 0:
                continue
            nb = pad[hh + dy:hh + dy + H, hw + dx:hw + dx + W]
            code |= (nb < Y).astype(np.uint64) << np.uint64(k)
            k += 1
    return code


def arms_cumprod(rgb, L1=17, tau1=20):
    """Arm lengths as the count of leading passes of the colour test."""
    I = rgb.astype(np.int64)
    H, W = I.shape[:2]
    out = np.zeros((H, W, 4), dtype=np.uint8)
    for k, (ex, ey) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
        alive = np.ones((H, W), dtype=bool)
        count = np.zeros((H, W), dtype=np.int64)
        for j in range(1, L1 + 1):
            ys, xs = np.mgrid[0:H, 0:W]
            nx, ny = xs + j * ex, ys + j * ey
            inside = (nx >= 0) & (nx < W) & (ny >= 0) & (ny < H)
            nxc, nyc = np.clip(nx, 0, W - 1), np.clip(ny, 0, H - 1)
            diff = np.abs(I[nyc, nxc] - I).max(axis=2)
            alive &= inside & (diff < tau1)
            count += alive
        out[..., k] = count
    return out


def popcount64(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a.ravel()]).reshape(a.shape)


def cost_real(ref, L, R, cL, cR, arms_ref, D, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0):
    """Eq. 1 in float64, partner outside the image -> 1.0.  D x H x W."""
    I0, I1 = (L, R) if ref == 0 else (R, L)
    C0, C1 = (cL, cR) if ref == 0 else (cR, cL)
    H, W = L.shape[:2]
    lmin = arms_ref.min(axis=2).astype(np.float64)
    alpha = 1.0 - np.exp(-gamma / (lmin + eps))
    out = np.ones((D, H, W))
    for d in range(D):
        for x in range(W):
            xo = x - d if ref == 0 else x + d
            if xo < 0 or xo >= W:
                continue
            s = np.abs(I0[:, x].astype(np.int64) - I1[:, xo].astype(np.int64)).sum(axis=1)
            h = popcount64(C0[:, x] ^ C1[:, xo])
            out[d, :, x] = (alpha[:, x] * (1.0 - np.exp(-(s / 3.0) / lam_ad))
                            + (1.0 - alpha[:, x]) * (1.0 - np.exp(-h / lam_c)))
    return out


def region1(arms, x, y):
    """Stage-1 cross region of p: horizontal segments of the pixels on p's vertical arm."""
    l, r, u, dn = (int(v) for v in arms[y, x])
    pts = []
    for yy in range(y - u, y + dn + 1):
        la, ra = int(arms[yy, x, 0]), int(arms[yy, x, 1])
        pts.extend((xx, yy) for xx in range(x - la, x + ra + 1))
    return pts


def region2(arms, x, y):
    """Stage-2 cross region of p: vertical segments of the pixels on p's horizontal arm."""
    l, r, u, dn = (int(v) for v in arms[y, x])
    pts = []
    for xx in range(x - l, x + r + 1):
        ua, da = int(arms[y, xx, 2]), int(arms[y, xx, 3])
        pts.extend((xx, yy) for yy in range(y - ua, y + da + 1))
    return pts


def aggregate_sets(q, arms, iters=2):
    """Two-stage fixed-point aggregation by explicit region enumeration."""
    D, H, W = q.shape
    R1 = [[region1(arms, x, y) for x in range(W)] for y in range(H)]
    R2 = [[region2(arms, x, y) for x in range(W)] for y in range(H)]
    out = np.empty((D, H, W), dtype=np.float32)
    for d in range(D):
        qd = q[d].astype(np.int64)
        a1 = np.empty((H, W), dtype=np.int64)
        for y in range(H):
            for x in range(W):
                pts = R1[y][x]
                s = sum(int(qd[yy, xx]) for xx, yy in pts)
                n = len(pts)
                if iters == 1:
                    out[d, y, x] = np.float32(np.float32(s) / np.float32(n)) * np.float32(2.0 ** -20)
                else:
                    a1[y, x] = (s + n // 2) // n
        if iters == 1:
            continue
        for y in range(H):
            for x in range(W):
                pts = R2[y][x]
                s = sum(int(a1[yy, xx]) for xx, yy in pts)
                n = len(pts)
                out[d, y, x] = np.float32(np.float32(s) / np.float32(n)) * np.float32(2.0 ** -20)
    return out


def aggregate_real(c, arms, iters=2):
    """Real-valued Eq. 2 (applied once or twice) by region enumeration."""
    D, H, W = c.shape
    R1 = [[region1(arms, x, y) for x in range(W)] for y in range(H)]
    R2 = [[region2(arms, x, y) for x in range(W)] for y in range(H)]
    out = np.empty((D, H, W))
    for d in range(D):
        a1 = np.empty((H, W))
        for y in range(H):
            for x in range(W):
                pts = R1[y][x]
                a1[y, x] = sum(c[d, yy, xx] for xx, yy in pts) / len(pts)
        if iters == 1:
            out[d] = a1
            continue
        for y in range(H):
            for x in range(W):
                pts = R2[y][x]
                out[d, y, x] = sum(a1[yy, xx] for xx, yy in pts) / len(pts)
    return out


def soft_argmin(vol, T):
    """Soft-argmin over axis 0 of a D x H x W volume (float64)."""
    D = vol.shape[0]
    z = -vol / T
    z = z - z.max(axis=0, keepdims=True)
    w = np.exp(z)
    w /= w.sum(axis=0, keepdims=True)
    return (np.arange(D)[:, None, None] * w).sum(axis=0)


def box_mean_int(a, r):
    """Rounded (half-up) mean over the (2r+1)^2 square, valid interior only,
    by 2-D cumulative sums (a textbook box filter)."""
    a = a.astype(np.int64)
    H, W = a.shape
    S = np.zeros((H + 1, W + 1), dtype=np.int64)
    S[1:, 1:] = a.cumsum(0).cumsum(1)
    k = 2 * r + 1
    tot = S[k:, k:] - S[:-k, k:] - S[k:, :-k] + S[:-k, :-k]
    n = k * k
    return (tot + n // 2) // n


def alpha_closed(L, gamma=1.0, eps=0.8):
    return 1.0 - math.exp(-gamma / (L + eps))


# ---------------------------------------------------------------------------
# Depth contour filter (Sec. 5), written with whole-array shifts
# ---------------------------------------------------------------------------

def flow_terms_ref(F):
    """Amplitude (Eq. 6-8) and score (Eq. 9-11) of one flow field, float32,
    as array expressions: neighbours by slicing, p0 / p1 by fancy indexing."""
    F = np.asarray(F, np.float32)
    U, V = F[..., 0], F[..., 1]
    h, w = U.shape
    r = np.sqrt(U * U + V * V)                       # float32, correctly rounded
    gu = np.zeros_like(r)
    gv = np.zeros_like(r)
    gu[:, :-1] = np.abs(r[:, 1:] - r[:, :-1])
    gv[:-1, :] = np.abs(r[1:, :] - r[:-1, :])
    M = np.maximum(gu, gv)
    with np.errstate(divide="ignore", invalid="ignore"):
        ex = np.where(r > 0, U / r, np.float32(0)).astype(np.float32)
        ey = np.where(r > 0, V / r, np.float32(0)).astype(np.float32)
    sx, sy = np.rint(ex).astype(int), np.rint(ey).astype(int)
    ys, xs = np.mgrid[0:h, 0:w]
    x1, y1 = np.clip(xs + sx, 0, w - 1), np.clip(ys + sy, 0, h - 1)
    x0, y0 = np.clip(xs - sx, 0, w - 1), np.clip(ys - sy, 0, h - 1)
    f1 = U[y1, x1] * ex + V[y1, x1] * ey
    f0 = U[y0, x0] * ex + V[y0, x0] * ey
    S = np.where(r > 0, f1 - f0, np.float32(0)).astype(np.float32)
    return M, S


def flow_fuse_ref(past, future, R=2):
    """Eq. 12 (larger score wins; equal scores keep the larger amplitude),
    the clipped (2R+1)^2 window mean in float64, and the division by the
    maximum.  Agrees with the oracle to float32 rounding of the window sums."""
    Mp, Sp = flow_terms_ref(past)
    Mf, Sf = flow_terms_ref(future)
    fu = np.where(Sp > Sf, Mp, np.where(Sf > Sp, Mf, np.maximum(Mp, Mf))).astype(np.float64)
    h, w = fu.shape
    pad = np.pad(fu, R)
    one = np.pad(np.ones((h, w)), R)
    s = np.zeros((h, w))
    n = np.zeros((h, w))
    for dy in range(2 * R + 1):
        for dx in range(2 * R + 1):
            s += pad[dy:dy + h, dx:dx + w]
            n += one[dy:dy + h, dx:dx + w]
    box = s / n
    return box / box.max() if box.max() > 0 else np.zeros_like(box)


def contour_ref(Y, Mn, Thigh=0.06, Tlow=0.03, Tdepth=0.03):
    """Gated Canny of Sec. 5.3 with the readings of the oracle, as array
    operations: Sobel by shifted copies of the edge-padded image, the sector
    of every pixel, suppression by gathering the two neighbours, and
    hysteresis as 8-connected component labelling (scipy)."""
    from scipy import ndimage
    Y = np.asarray(Y, np.int64)
    H, W = Y.shape
    pad = np.pad(Y, 1, mode="edge")

    def at(dx, dy):
        return pad[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]

    gx = (at(1, -1) + 2 * at(1, 0) + at(1, 1)) - (at(-1, -1) + 2 * at(-1, 0) + at(-1, 1))
    gy = (at(-1, 1) + 2 * at(0, 1) + at(1, 1)) - (at(-1, -1) + 2 * at(0, -1) + at(1, -1))
    G2 = gx * gx + gy * gy
    mx = int(G2.max())
    ax, ay = np.abs(gx), np.abs(gy)
    horiz = 128 * ay < 53 * ax
    vert = ~horiz & (128 * ax < 53 * ay)
    same = (gx > 0) == (gy > 0)
    dx = np.where(horiz, 1, np.where(vert, 0, 1))
    dy = np.where(horiz, 0, np.where(vert, 1, np.where(same, 1, -1)))
    ys, xs = np.mgrid[0:H, 0:W]
    G2p = np.pad(G2, 1)                                  # 0 outside the image
    before = G2p[1 + ys - dy, 1 + xs - dx]
    after = G2p[1 + ys + dy, 1 + xs + dx]
    keep = (G2 > before) & (G2 >= after)
    h, w = Mn.shape
    Mn = np.asarray(Mn, np.float32)
    gate = Mn[np.minimum(ys // 2, h - 1), np.minimum(xs // 2, w - 1)] >= np.float32(Tdepth)
    keep &= gate
    v = G2.astype(np.float64)
    th, tl = float(np.float32(Thigh)), float(np.float32(Tlow))   # float parameters
    strong = keep & (v > th * th * mx)
    weak = keep & (v > tl * tl * mx)
    lab, n = ndimage.label(weak, structure=np.ones((3, 3)))
    on = np.zeros(n + 1, bool)
    on[np.unique(lab[strong])] = True
    on[0] = False
    B = on[lab].astype(np.uint8)
    MI = (np.sqrt((v / mx).astype(np.float32)) if mx > 0 else np.zeros((H, W), np.float32))
    return B, MI
