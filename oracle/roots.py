"""Step (ii) of syndrome decoding: roots of the locator polynomial
P(z) = z^a + c_{a-1} z^{a-1} + ... + c_0  (Sec. II-B, Eq. (4)) by the
closed forms of the paper's Appendix, for a <= 4.

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle/__init__.py).

The printed Appendix has typos; the corrected readings used here are:
  * a = 3 (Cardano): A is a cube root of Q - sqrt(Q^2 + P^3) with
    Q = c0/2 - c1 c2/6 + c2^3/27 and P = c1/3 - c2^2/9; B = -P/A is taken from
    the same branch of A.  Of the six (sign, cube-root branch) choices the one
    with the largest |A| is used, so that B = -P/A is well conditioned.
  * a = 4 (Ferrari): the factorisation
    (z^2 + (c3/2 + A) z + Y + B)(z^2 + (c3/2 - A) z + Y - B) needs
    B = (c3 Y - c1) / (2 A) (the Appendix prints a denominator of A).  Y comes
    from the resolvent cubic through C = cbrt(G + sqrt(G^2 + H^3)), D = -H/C,
    Y = c2/6 - C - D; the branch with the largest |A| is used (the principal
    branch can give A = 0, e.g. for biquadratic polynomials).
Each root then gets one Newton step on P itself.

Precision limit: like any route from the coefficients, the closed forms
lose accuracy on clusters of adjacent grid roots; four adjacent roots of
unity at d >= 4096 come out with errors near the grid spacing (three
adjacent ones stay below 1e-10), so such a bin is rejected by the grid check.
"""
from __future__ import annotations

import numpy as np

W1 = complex(-0.5, np.sqrt(3.0) / 2.0)   # cube roots of unity (Appendix, a = 3)
W2 = complex(-0.5, -np.sqrt(3.0) / 2.0)


def _cbrt_all(w: complex):
    r = complex(w) ** (1.0 / 3.0) if w != 0 else 0j
    return (r, r * W1, r * W2)


def _poly_eval(c, z):
    """P(z) and P'(z) for monic P with low-order-first coefficients c."""
    a = len(c)
    p = 1.0 + 0j
    dp = 0j
    for j in range(a - 1, -1, -1):
        dp = dp * z + p
        p = p * z + c[j]
    return p, dp


def _newton_polish(c, zs):
    out = []
    for z in zs:
        p, dp = _poly_eval(c, z)
        if dp != 0 and np.isfinite(p) and np.isfinite(dp):
            z = z - p / dp
        out.append(complex(z))
    return out


def roots_a1(c):
    return [complex(-c[0])]


def roots_a2(c):
    c0, c1 = complex(c[0]), complex(c[1])
    s = np.sqrt(c1 * c1 - 4.0 * c0 + 0j)
    return [0.5 * (-c1 - s), 0.5 * (-c1 + s)]


def roots_a3(c):
    c0, c1, c2 = (complex(v) for v in c)
    q = c0 / 2.0 - c1 * c2 / 6.0 + c2 ** 3 / 27.0
    p = c1 / 3.0 - c2 ** 2 / 9.0
    disc = np.sqrt(q * q + p ** 3 + 0j)
    best = 0j
    for sgn in (1.0, -1.0):
        for a_ in _cbrt_all(q - sgn * disc):
            if abs(a_) > abs(best):
                best = a_
    shift = -c2 / 3.0
    if best == 0:
        return [shift, shift, shift]
    a_ = best
    b_ = -p / a_
    return [shift - a_ - b_, shift - W1 * a_ - W2 * b_, shift - W2 * a_ - W1 * b_]


def roots_a4(c):
    c0, c1, c2, c3 = (complex(v) for v in c)
    h = (3.0 * c1 * c3 - 12.0 * c0 - c2 * c2) / 36.0
    g = (72.0 * c0 * c2 + 9.0 * c1 * c2 * c3 - 27.0 * c1 * c1
         - 27.0 * c0 * c3 * c3 - 2.0 * c2 ** 3) / 432.0
    disc = np.sqrt(g * g + h ** 3 + 0j)
    best_a, best_y = None, None
    for sgn in (1.0, -1.0):
        for cb in _cbrt_all(g + sgn * disc):
            if cb == 0:
                if h != 0:
                    continue
                y = c2 / 6.0
            else:
                y = c2 / 6.0 - cb - (-h / cb)
            a_ = 0.5 * np.sqrt(c3 * c3 - 4.0 * c2 + 8.0 * y + 0j)
            if best_a is None or abs(a_) > abs(best_a):
                best_a, best_y = a_, y
    a_, y = best_a, best_y
    if abs(a_) == 0.0:
        b_ = np.sqrt(y * y - c0 + 0j)       # Y^2 - B^2 = c0 when the linear term vanishes
    else:
        b_ = (c3 * y - c1) / (2.0 * a_)
    u, v = c3 / 2.0 + a_, c3 / 2.0 - a_
    su = np.sqrt(u * u - 4.0 * (y + b_) + 0j)
    sv = np.sqrt(v * v - 4.0 * (y - b_) + 0j)
    return [0.5 * (-u - su), 0.5 * (-u + su), 0.5 * (-v - sv), 0.5 * (-v + sv)]


_CLOSED = {1: roots_a1, 2: roots_a2, 3: roots_a3, 4: roots_a4}


def poly_roots(c):
    """All a roots of z^a + sum_j c_j z^j (a = len(c) <= 4), closed form + one Newton step."""
    a = len(c)
    if a not in _CLOSED:
        raise ValueError("closed forms exist for a <= 4 only")
    with np.errstate(all="ignore"):
        zs = _CLOSED[a](c)
        return _newton_polish(c, zs)
