"""The paper's lifting schemes written in its 2x2-polyphase matrix notation (FP64).

TEST INFRASTRUCTURE (part of the oracle). Used to pin the form agreement of
the separable and non-separable schemes and the step and operation counts of
Table 1. Slow and plain: whole-array numpy operations, one per term.

Notation (Sec. 2-3). A 2x2 block of pixels at quad (i, j) holds the four
polyphase components 1..4, here a = x[2j, 2i], b = x[2j, 2i+1],
c = x[2j+1, 2i], d = x[2j+1, 2i+1]. m is the horizontal axis, n the vertical
one. A lifting filter F(z) acts along m; its transpose F* acts along n.

  separable lifting, per pair:  S_U^V | S_U^H | T_P^V | T_P^H |
      T_P^H: b += P a,  d += P c          T_P^V: c += P* a, d += P* b
      S_U^H: a += U b,  c += U d          S_U^V: a += U* c, b += U* d
  non-separable lifting, per pair:  S_U | T_P |
      T_P:  b += P a;  c += P* a;  d += P P* a + P* b + P c   (pre-step values)
      S_U:  a += U b + U* c + U U* d;  b += U* d;  c += U d   (pre-step values)

The constant split (Sec. 3): P = P0 + P1 and U = U0 + U1 where P0, U0 are the
zero-delay taps. The non-separable step keeps only P1 (U1); the P0 (U0) part
then runs as separable H and V steps on the unit's own quad with no barrier.

Lifting filters (reading of the paper, which does not print them): the
predict adds the even neighbours of an odd sample, P(z) = p (1 + z), i.e.
P0 = p and P1 = p z (the right or lower neighbour); the update adds the odd
neighbours of an even sample, U(z) = u (1 + 1/z), i.e. U0 = u and U1 = u/z
(the left or upper neighbour). Lifting pairs and scaling are restated here
from the standard CDF factorisation and are pinned, with the C oracle, by the
closed-form filter tests.

Boundaries: 'symmetric' (whole-sample symmetric extension: a neighbour index
past the last quad maps to the last quad, one before the first quad maps to
the first) or 'periodic' (used only to compare against the matrices in the
z-domain).
"""
from __future__ import annotations

import numpy as np

CDF97_PAIRS = ((-1.586134342059924, -0.052980118572961),
               (0.882911075530934, 0.443506852043971))
CDF97_K = 1.230174104914001
CDF53_PAIRS = ((-0.5, 0.25),)


def wavelet_def(wavelet: str):
    """(pairs, low scale, high scale) for 'cdf97' or 'cdf53'."""
    if wavelet == "cdf97":
        return CDF97_PAIRS, 1.0 / CDF97_K, CDF97_K / 2.0
    if wavelet == "cdf53":
        return CDF53_PAIRS, 1.0, 0.5
    raise ValueError(wavelet)


class OpCounter:
    """Counts multiply-accumulates per quad, one per term added to a component."""

    def __init__(self):
        self.macs = 0
        self.steps = 0

    def mac(self, dst, coef, src):
        self.macs += 1
        return dst + coef * src


def _shift(f, dm, dn, boundary):
    """Neighbour view g[j, i] = f[j + dn, i + dm] with the boundary rule."""
    if boundary == "periodic":
        return np.roll(f, shift=(-dn, -dm), axis=(0, 1))
    ny, nx = f.shape
    ii = np.clip(np.arange(nx) + dm, 0, nx - 1)
    jj = np.clip(np.arange(ny) + dn, 0, ny - 1)
    return f[np.ix_(jj, ii)]


def split_quads(x):
    x = np.asarray(x, dtype=np.float64)
    return [x[0::2, 0::2].copy(), x[0::2, 1::2].copy(),
            x[1::2, 0::2].copy(), x[1::2, 1::2].copy()]


def merge_quads(q):
    a, b, c, d = q
    ny, nx = a.shape
    x = np.empty((2 * ny, 2 * nx))
    x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2] = a, b, c, d
    return x


# ---- separable steps (T^H, T^V, S^H, S^V), each term one MAC ---------------

def sep_predict_h(q, p, ops, bnd):
    a, b, c, d = q
    b = ops.mac(ops.mac(b, p, a), p, _shift(a, 1, 0, bnd))
    d = ops.mac(ops.mac(d, p, c), p, _shift(c, 1, 0, bnd))
    return [a, b, c, d]


def sep_predict_v(q, p, ops, bnd):
    a, b, c, d = q
    c = ops.mac(ops.mac(c, p, a), p, _shift(a, 0, 1, bnd))
    d = ops.mac(ops.mac(d, p, b), p, _shift(b, 0, 1, bnd))
    return [a, b, c, d]


def sep_update_h(q, u, ops, bnd):
    a, b, c, d = q
    a = ops.mac(ops.mac(a, u, b), u, _shift(b, -1, 0, bnd))
    c = ops.mac(ops.mac(c, u, d), u, _shift(d, -1, 0, bnd))
    return [a, b, c, d]


def sep_update_v(q, u, ops, bnd):
    a, b, c, d = q
    a = ops.mac(ops.mac(a, u, c), u, _shift(c, 0, -1, bnd))
    b = ops.mac(ops.mac(b, u, d), u, _shift(d, 0, -1, bnd))
    return [a, b, c, d]


# ---- non-separable steps ---------------------------------------------------

def nonsep_predict_full(q, p, ops, bnd):
    """T_P with the whole polynomial P = p(1+z) in the spatial step."""
    a, b, c, d = q
    ar, ad, adr = _shift(a, 1, 0, bnd), _shift(a, 0, 1, bnd), _shift(a, 1, 1, bnd)
    nb = ops.mac(ops.mac(b, p, a), p, ar)                        # P a
    nc = ops.mac(ops.mac(c, p, a), p, ad)                        # P* a
    nd = d
    for t in (a, ar, ad, adr):                                   # P P* a
        nd = ops.mac(nd, p * p, t)
    nd = ops.mac(ops.mac(nd, p, b), p, _shift(b, 0, 1, bnd))     # P* b
    nd = ops.mac(ops.mac(nd, p, c), p, _shift(c, 1, 0, bnd))     # P c
    return [a, nb, nc, nd]


def nonsep_update_full(q, u, ops, bnd):
    """S_U with the whole polynomial U = u(1+1/z) in the spatial step."""
    a, b, c, d = q
    na = ops.mac(ops.mac(a, u, b), u, _shift(b, -1, 0, bnd))     # U b
    na = ops.mac(ops.mac(na, u, c), u, _shift(c, 0, -1, bnd))    # U* c
    for t in (d, _shift(d, -1, 0, bnd), _shift(d, 0, -1, bnd),
              _shift(d, -1, -1, bnd)):                           # U U* d
        na = ops.mac(na, u * u, t)
    nb = ops.mac(ops.mac(b, u, d), u, _shift(d, 0, -1, bnd))     # U* d
    nc = ops.mac(ops.mac(c, u, d), u, _shift(d, -1, 0, bnd))     # U d
    return [na, nb, nc, d]


def nonsep_predict_split(q, p, ops, bnd):
    """T_P as the spatial T_{P1} (neighbours only) followed by the separable
    P0 steps on the unit's own quad (H then V)."""
    a, b, c, d = q
    # T_{P1}: P1 = p z reads the right / lower neighbour; pre-step values.
    nb = ops.mac(b, p, _shift(a, 1, 0, bnd))
    nc = ops.mac(c, p, _shift(a, 0, 1, bnd))
    nd = ops.mac(d, p, _shift(c, 1, 0, bnd))
    nd = ops.mac(nd, p, _shift(b, 0, 1, bnd))
    nd = ops.mac(nd, p * p, _shift(a, 1, 1, bnd))
    # T^H_{P0} then T^V_{P0}, own quad only.
    nb = ops.mac(nb, p, a)
    nd = ops.mac(nd, p, nc)
    nc = ops.mac(nc, p, a)
    nd = ops.mac(nd, p, nb)
    return [a, nb, nc, nd]


def nonsep_update_split(q, u, ops, bnd):
    """S_U as the spatial S_{U1} followed by the separable U0 steps."""
    a, b, c, d = q
    # S_{U1}: U1 = u/z reads the left / upper neighbour; pre-step values.
    na = ops.mac(a, u, _shift(b, -1, 0, bnd))
    na = ops.mac(na, u, _shift(c, 0, -1, bnd))
    na = ops.mac(na, u * u, _shift(d, -1, -1, bnd))
    nb = ops.mac(b, u, _shift(d, 0, -1, bnd))
    nc = ops.mac(c, u, _shift(d, -1, 0, bnd))
    # S^H_{U0} then S^V_{U0}, own quad only.
    na = ops.mac(na, u, nb)
    nc = ops.mac(nc, u, d)
    na = ops.mac(na, u, nc)
    nb = ops.mac(nb, u, d)
    return [na, nb, nc, d]


SCHEMES = ("separable", "nonseparable", "nonseparable_full")


def _pair_steps(scheme):
    """The barrier-separated steps of one lifting pair, in execution order."""
    if scheme == "separable":
        return [("P", sep_predict_h), ("P", sep_predict_v),
                ("U", sep_update_h), ("U", sep_update_v)]
    if scheme == "nonseparable":
        return [("P", nonsep_predict_split), ("U", nonsep_update_split)]
    if scheme == "nonseparable_full":
        return [("P", nonsep_predict_full), ("U", nonsep_update_full)]
    raise ValueError(scheme)


def forward_level(x, wavelet="cdf97", scheme="nonseparable", ops=None,
                  boundary="symmetric"):
    """One level: returns the quads (LL, HL, LH, HH) as four arrays."""
    pairs, zl, zh = wavelet_def(wavelet)
    ops = ops or OpCounter()
    q = split_quads(x)
    for p, u in pairs:
        for kind, step in _pair_steps(scheme):
            q = step(q, p if kind == "P" else u, ops, boundary)
            ops.steps += 1
    a, b, c, d = q
    return [a * zl * zl, b * zl * zh, c * zh * zl, d * zh * zh]


def inverse_level(bands, wavelet="cdf97", scheme="nonseparable", ops=None,
                  boundary="symmetric"):
    """Inverse of :func:`forward_level`: each step undone with negated
    coefficients, steps and pairs in reverse order."""
    pairs, zl, zh = wavelet_def(wavelet)
    ops = ops or OpCounter()
    ll, hl, lh, hh = bands
    q = [ll / (zl * zl), hl / (zl * zh), lh / (zh * zl), hh / (zh * zh)]
    for p, u in reversed(pairs):
        for kind, step in reversed(_pair_steps(scheme)):
            q = step(q, -(p if kind == "P" else u), ops, boundary)
            ops.steps += 1
    return merge_quads(q)


def forward(x, wavelet="cdf97", levels=1, scheme="nonseparable"):
    """L-level forward DWT, Mallat layout, by the chosen scheme."""
    out = np.array(x, dtype=np.float64, copy=True)
    H, W = out.shape
    for j in range(levels):
        h, w = H >> j, W >> j
        ll, hl, lh, hh = forward_level(out[:h, :w], wavelet, scheme)
        out[:h // 2, :w // 2] = ll
        out[:h // 2, w // 2:w] = hl
        out[h // 2:h, :w // 2] = lh
        out[h // 2:h, w // 2:w] = hh
    return out


def inverse(c, wavelet="cdf97", levels=1, scheme="nonseparable"):
    out = np.array(c, dtype=np.float64, copy=True)
    H, W = out.shape
    for j in reversed(range(levels)):
        h, w = H >> j, W >> j
        bands = [out[:h // 2, :w // 2], out[:h // 2, w // 2:w],
                 out[h // 2:h, :w // 2], out[h // 2:h, w // 2:w]]
        out[:h, :w] = inverse_level([b.copy() for b in bands], wavelet, scheme)
    return out


# ---- the step matrices of Sec. 2-3, evaluated at a point (z_m, z_n) ---------

def step_matrices(p, u, zm, zn):
    """The 4x4 polyphase step matrices at (z_m, z_n) for P = p(1+z), U = u(1+1/z).

    Acting on the column (a, b, c, d); the matrix of a later step multiplies
    on the left.
    """
    P, Ps = p * (1 + zm), p * (1 + zn)
    U, Us = u * (1 + 1 / zm), u * (1 + 1 / zn)
    I = np.eye(4, dtype=complex)
    TPH = I.copy(); TPH[1, 0] = P; TPH[3, 2] = P
    TPV = I.copy(); TPV[2, 0] = Ps; TPV[3, 1] = Ps
    SUH = I.copy(); SUH[0, 1] = U; SUH[2, 3] = U
    SUV = I.copy(); SUV[0, 2] = Us; SUV[1, 3] = Us
    TP = I.copy()
    TP[1, 0] = P; TP[2, 0] = Ps; TP[3, 0] = P * Ps; TP[3, 1] = Ps; TP[3, 2] = P
    SU = I.copy()
    SU[0, 1] = U; SU[0, 2] = Us; SU[0, 3] = U * Us; SU[1, 3] = Us; SU[2, 3] = U
    return dict(TPH=TPH, TPV=TPV, SUH=SUH, SUV=SUV, TP=TP, SU=SU)
