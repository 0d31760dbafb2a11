"""The squared cosines of the float32 path's second attempt (§5, (5.1)-(5.2),
(5.20)-(5.25)), restated in numpy.

Where the general branch's result fails the check, the kernel forms new
squared cosines v = cos^2 phi2, w = cos^2 phi3 and runs the general branch's
angle selection on them:
  - near a double root, v = ||row 1||^2 / (||row 1||^2 + ||row 2||^2 +
    ||row 3||^2) for the rows of A - lm I (lm the mean of the close pair), and
    w = 1 for an isolated maximum, 0 for an isolated minimum;
  - for a diagonal matrix, v and w in {0, 1} from the slot of A11.
These CPU tests check the algebra those choices rest on: the row-norm
quotient equals u1^2 for the isolated eigenvector u and equals 1 minus the
paper's (5.21) quantity (A11 - ls)/(lm - ls) at an exact double root; it
stays within the square of the relative split of u1^2 near one; and the
first row of D in the slot order (max, min, mid) has the squared entries
that (5.1)-(5.2) turn into these v and w.
"""

import numpy as np


def _rot(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    return q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]


def _row_norm_v(A, lm):
    B = A - lm[:, None, None] * np.eye(3)
    r = np.sum(B * B, axis=2)            # squared norms of the three rows
    return r[:, 0] / r.sum(axis=1)


def test_row_norm_quotient_is_u1_squared_and_5_21():
    rng = np.random.default_rng(21)
    n = 2000
    Q = _rot(rng, n)
    u = Q[:, :, 0]                        # isolated unit eigenvector
    lm = rng.uniform(-1, 1, n)
    ls = lm + np.where(rng.random(n) < 0.5, -1, 1) * rng.uniform(0.1, 1.0, n)
    A = lm[:, None, None] * np.eye(3) + (ls - lm)[:, None, None] * u[:, :, None] * u[:, None, :]
    v = _row_norm_v(A, lm)
    assert np.abs(v - u[:, 0] ** 2).max() < 1e-13
    # (5.21), paper's column order (u third): cos^2 phi2 = (A11 - ls)/(lm - ls) = 1 - u1^2
    c521 = (A[:, 0, 0] - ls) / (lm - ls)
    assert np.abs((1.0 - v) - c521).max() < 1e-12


def test_row_norm_quotient_near_a_double_root():
    """With the pair split by delta, A - lm I gains (delta/2)(p p^T - q q^T)
    for the pair's eigenvectors p, q, which adds (delta/2)^2 (p1^2 + q1^2) to
    row 1's squared norm and nothing at first order: v stays within
    (delta / (ls - lm))^2 of u1^2."""
    rng = np.random.default_rng(22)
    n = 2000
    Q = _rot(rng, n)
    lm = rng.uniform(-1, 1, n)
    gap = rng.uniform(0.1, 1.0, n)
    ls = lm + gap
    for rel in (1e-7, 1e-5, 1e-3):
        delta = rel * gap
        lam = np.stack([ls, lm - 0.5 * delta, lm + 0.5 * delta], axis=1)
        A = np.einsum("nik,nk,njk->nij", Q, lam, Q)
        v = _row_norm_v(A, lm)
        err = np.abs(v - Q[:, 0, 0] ** 2)
        assert np.all(err <= 0.5 * rel ** 2 + 1e-14), (rel, err.max())


def test_slot_order_first_row_gives_v_and_w():
    """D in the slot order (max, min, mid).  (5.1)-(5.2): v = D11^2 + D12^2,
    w = D11^2 / (D11^2 + D12^2) (w = 1 when v = 0).  Isolated maximum (u in
    column 0) with the pair's basis chosen so that D12 = 0: v = u1^2, w = 1.
    Isolated minimum (u in column 1) with D11 = 0: v = u1^2, w = 0.  A
    diagonal matrix: the first row is the axis of A11's slot."""
    rng = np.random.default_rng(23)
    for iso in ("max", "min"):
        for _ in range(200):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            # the pair's plane, with a basis vector orthogonal to e1 where possible
            a = np.cross(u, [1.0, 0.0, 0.0])
            a /= np.linalg.norm(a)               # a1 = 0
            b = np.cross(u, a)
            cols = [u, a, b] if iso == "max" else [a, u, b]   # D12 = a1 = 0, or D11 = a1 = 0
            D = np.stack(cols, axis=1)
            v = D[0, 0] ** 2 + D[0, 1] ** 2
            w = D[0, 0] ** 2 / v if v > 0 else 1.0
            assert abs(v - u[0] ** 2) < 1e-14
            assert abs(w - (1.0 if iso == "max" else 0.0)) < 1e-14
    for d in ([3.0, 1.0, 2.0], [1.0, 3.0, 2.0], [2.0, 3.0, 1.0], [2.0, 2.0, 1.0], [1.0, 2.0, 1.0]):
        d = np.array(d)
        order = [int(np.argmax(d)), int(np.argmin(d))]
        order.append(3 - sum(order))
        D = np.eye(3)[:, order]                   # columns: axes of max, min, mid
        v = D[0, 0] ** 2 + D[0, 1] ** 2
        w = D[0, 0] ** 2 / v if v > 0 else 1.0
        top, bottom = d[0] == d.max(), d[0] != d.max() and d[0] == d.min()
        assert v == (1.0 if (top or bottom) else 0.0)
        assert w == (0.0 if bottom else 1.0)
