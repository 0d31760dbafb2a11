"""The sign selection of the HIP path against the paper's rule (§5, (5.11)-(5.15)).

The kernels do not compare four arctangents.  They take the sign of the
product sin(phi2) sin(phi3) from
    K = A12 A13 (A22 - A33) - A23 (A12^2 - A13^2),
using the identity (derived from (5.5)-(5.8) with cos^2 + sin^2 = 1)
    Re(z+^2 conj z+) - Re(z-^2 conj z-) = 8 K G12 G13 G32 c2^2 c3 s2 s3,
where z1 = conj(f1) g1 and z2 = conj(f2) g2 for the two products, and then the
overall sign from the principal square root of z2.  These CPU tests restate
the identity in numpy on random values, and check on the oracle (which applies
the paper's smallest-distance rule to the four combinations) that the product
it chooses is sign(K) wherever its choice is clear.
"""

import numpy as np

import oracle
import synth


def _scores(a12, a13, a22, a33, a23, G12, G13, G32, v, w):
    s2sq, cw = 1.0 - v, 1.0 - w
    c2, s2, c3, s3 = np.sqrt(v), np.sqrt(s2sq), np.sqrt(w), np.sqrt(cw)
    al = G12 * c2 * s3 * c3
    be = (G13 * w - G32 * cw) * s2 * c2
    ga = G12 * (cw - w * s2sq) - G32 * v
    de = 2.0 * G12 * s2 * s3 * c3
    F1 = a12 + 1j * a13                  # conj(f1), (5.5)
    F2 = (a22 - a33) + 2j * a23          # conj(f2), (5.6)
    out = []
    for t in (1.0, -1.0):                # product s2 s3
        z1 = F1 * (t * al + 1j * be)
        z2 = F2 * (ga + 1j * t * de)
        out.append(np.real(z1 * z1 * np.conj(z2)))
    return out[0], out[1], 8.0 * G12 * G13 * G32 * v * c3 * s2 * s3


def _key(a12, a13, a22, a33, a23):
    return a12 * a13 * (a22 - a33) - a23 * (a12 * a12 - a13 * a13)


def test_product_identity_random_values():
    rng = np.random.default_rng(5)
    n = 20000
    a12, a13, a22, a33, a23 = rng.uniform(-1, 1, (5, n))
    G13, G32 = rng.uniform(0, 2, (2, n))
    G12 = G13 + G32
    v, w = rng.uniform(0, 1, (2, n))
    Cp, Cm, X = _scores(a12, a13, a22, a33, a23, G12, G13, G32, v, w)
    K = _key(a12, a13, a22, a33, a23)
    scale = np.abs(Cp) + np.abs(Cm) + 1.0
    assert np.all(np.abs((Cp - Cm) - K * X) <= 1e-13 * scale)
    assert np.all(X >= 0)


def _product_of(chosen):
    # combinations in the order (+,+), (+,-), (-,+), (-,-) of (sign phi2, sign phi3)
    return np.where((chosen == 0) | (chosen == 3), 1.0, -1.0)


def test_oracle_choice_matches_key():
    P = np.concatenate([synth.make_plain(1500, 16, seed=3)["planes3"],
                        synth.make_precision(1500, seed=11).astype(np.float64)], axis=1)
    checked = 0
    for j in range(P.shape[1]):
        d = oracle.eig3_debug(P[:, j])
        if d["branch"] != 0:
            continue
        delta = np.array(d["delta"])
        best_plus, best_minus = min(delta[0], delta[3]), min(delta[1], delta[2])
        if abs(best_plus - best_minus) < 1e-6:
            continue                     # both products fit: the choice is free
        a11, a22, a33, a12, a13, a23 = P[:, j]
        K = _key(a12, a13, a22, a33, a23)
        assert (K >= 0) == (_product_of(np.array(d["chosen"])) > 0), (j, K, delta)
        checked += 1
    assert checked > 2000
