"""Oracle of the depth densification (Sec. 6, Eq. 13-20) -- TEST INFRASTRUCTURE.

The dense depth D minimises, over every pixel p of an H x W grid,

    lambda_d  sum_p w_sparse(p) |D(p) - D_sparse(p)|^2                (Eq. 13, 14)
  + lambda_s  sum_p sum_{q in N4(p)} w_pq |D(p) - D(q)|^2              (Eq. 15-17)
  + lambda_s2 sum_p w_stable(p) |D(p) - D_pre(p)|^2                    (Eq. 18, 19)

(Eq. 20), with w_sparse = [D_sparse > 0], w_stable = [D_pre > 0] and
w_pq = 0 when exactly one of p, q is on the depth contour B_dp, else
max(1 - min(s_p, s_q), 0) with s = M_fuse * M_I.  The double sum visits
every 4-neighbour pair twice.  Setting the gradient to zero gives the sparse
symmetric system

    (lambda_d w_sparse + lambda_s2 w_stable + 2 lambda_s sum_q w_pq) D(p)
      - 2 lambda_s sum_q w_pq D(q) = lambda_d w_sparse D_sparse + lambda_s2 w_stable D_pre

READING (unanchored regions): pixels whose component of the graph of
w_pq > 0 edges holds no data or stability term do not determine D; they get
D = 0 (no depth, as in Eq. 14).  Everywhere else the system is positive
definite and is solved directly here (scipy's sparse LU), in float64.

Only the tests and the benchmark's CPU leg use this module.
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(lam_d=0.8, lam_s=1.2, lam_s2=0.02)  # Sec. 7.2


def edge_weights(Bdp, Mfuse, MI):
    """Eq. 16-17: (w_right, w_down), the weights of the edges (p, p + x) and
    (p, p + y); 0 on edges leaving the grid."""
    s = np.asarray(Mfuse, np.float64) * np.asarray(MI, np.float64)
    B = np.asarray(Bdp).astype(np.int64)
    H, W = B.shape
    wr = np.zeros((H, W))
    wd = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            for (yy, xx, out) in ((y, x + 1, wr), (y + 1, x, wd)):
                if yy >= H or xx >= W:
                    continue
                if B[y, x] + B[yy, xx] == 1:
                    out[y, x] = 0.0
                else:
                    out[y, x] = max(1.0 - min(s[y, x], s[yy, xx]), 0.0)
    return wr, wd


def system(Ds, Dpre, Bdp, Mfuse, MI, lam_d=0.8, lam_s=1.2, lam_s2=0.02):
    """The normal equations of Eq. 20 as (A, b) with A a scipy CSR matrix."""
    import scipy.sparse as sp
    Ds = np.asarray(Ds, np.float64)
    H, W = Ds.shape
    Dpre = np.zeros((H, W)) if Dpre is None else np.asarray(Dpre, np.float64)
    wsp = (Ds > 0).astype(np.float64)
    wst = (Dpre > 0).astype(np.float64)
    wr, wd = edge_weights(Bdp, Mfuse, MI)
    n = H * W
    idx = np.arange(n).reshape(H, W)
    diag = lam_d * wsp + lam_s2 * wst
    rows, cols, vals = [], [], []
    for w, (dy, dx) in ((wr, (0, 1)), (wd, (1, 0))):
        ys, xs = np.nonzero(w)
        p = idx[ys, xs]
        q = idx[ys + dy, xs + dx]
        c = 2.0 * lam_s * w[ys, xs]
        rows += [p, q]
        cols += [q, p]
        vals += [-c, -c]
        np.add.at(diag, (ys, xs), c)
        np.add.at(diag, (ys + dy, xs + dx), c)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    b = (lam_d * wsp * Ds + lam_s2 * wst * Dpre).ravel()
    anchor = (lam_d * wsp + lam_s2 * wst).ravel() > 0
    return A, b, anchor, (wr, wd)


def densify(Ds, Dpre, Bdp, Mfuse, MI, lam_d=0.8, lam_s=1.2, lam_s2=0.02):
    """Dense depth of Eq. 20 (float64, H x W)."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    import scipy.sparse.linalg as sla
    Ds = np.asarray(Ds, np.float64)
    H, W = Ds.shape
    A, b, anchor, _ = system(Ds, Dpre, Bdp, Mfuse, MI, lam_d, lam_s, lam_s2)
    off = A - sp.diags(A.diagonal())
    ncomp, label = cg.connected_components(off != 0, directed=False)
    keep = np.zeros(ncomp, bool)
    keep[np.unique(label[anchor])] = True
    live = keep[label]
    x = np.zeros(H * W)
    if live.any():
        sub = A[live][:, live].tocsc()
        x[live] = sla.spsolve(sub, b[live])
    return x.reshape(H, W)


def energy(D, Ds, Dpre, Bdp, Mfuse, MI, lam_d=0.8, lam_s=1.2, lam_s2=0.02):
    """Eq. 20's objective at D, summed term by term as printed."""
    D = np.asarray(D, np.float64)
    Ds = np.asarray(Ds, np.float64)
    H, W = D.shape
    Dpre = np.zeros((H, W)) if Dpre is None else np.asarray(Dpre, np.float64)
    s = np.asarray(Mfuse, np.float64) * np.asarray(MI, np.float64)
    B = np.asarray(Bdp).astype(np.int64)
    e = 0.0
    for y in range(H):
        for x in range(W):
            if Ds[y, x] > 0:
                e += lam_d * (D[y, x] - Ds[y, x]) ** 2
            if Dpre[y, x] > 0:
                e += lam_s2 * (D[y, x] - Dpre[y, x]) ** 2
            for (yy, xx) in ((y - 1, x), (y + 1, x), (y, x - 1), (y, x + 1)):
                if 0 <= yy < H and 0 <= xx < W:
                    if B[y, x] + B[yy, xx] == 1:
                        w = 0.0
                    else:
                        w = max(1.0 - min(s[y, x], s[yy, xx]), 0.0)
                    e += lam_s * w * (D[y, x] - D[yy, xx]) ** 2
    return e
