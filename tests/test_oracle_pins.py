"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these retypes the oracle's own formulas: the filter taps are derived
from the Daubechies polynomial, the boundary comes from numpy's reflect pad,
the counts from the paper's Table 1, and the rest are invariants (perfect
reconstruction, vanishing moments, constants, linearity, the z-domain matrices).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import filterbank as fb
from oracle import nonsep_model as nsm

WAVELETS = ["cdf53", "cdf97"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- closed-form filters ----------------------------------------------------

@pytest.mark.parametrize("w,nh,ng,vm", [("cdf53", 5, 3, 2), ("cdf97", 9, 7, 4)])
def test_closed_form_filter_properties(w, nh, ng, vm):
    h, g = fb.cdf_filters(w)
    assert h.size == nh and g.size == ng
    assert np.allclose(h, h[::-1]) and np.allclose(g, g[::-1])
    assert abs(h.sum() - 1.0) < 1e-14                       # DC gain 1
    k = np.arange(g.size) - g.size // 2
    assert abs(np.sum(g * (-1.0) ** k) - 1.0) < 1e-14       # Nyquist gain 1
    for m in range(vm):                                     # vanishing moments
        assert abs(np.sum(g * k.astype(float) ** m)) < 1e-13
    assert abs(np.sum(g * k.astype(float) ** vm)) > 1e-3
    # half-band product filter: analysis low x synthesis low has zero even
    # taps except the centre, which is 1/2 at unit DC gain
    syn = g * (-1.0) ** k
    prod = np.convolve(h, syn)
    c = prod.size // 2
    even = prod[c % 2::2]
    centre_idx = c // 2
    assert abs(even[centre_idx] - 0.5) < 1e-14
    assert np.all(np.abs(np.delete(even, centre_idx)) < 1e-14)


def test_cdf97_real_root_is_a_root():
    y = fb.daubechies_real_root()
    assert abs(1 + 4 * y + 10 * y * y + 20 * y ** 3) < 1e-14
    assert -0.35 < y < -0.33


# ---- 1-D oracle vs filter bank ------------------------------------------------

@pytest.mark.parametrize("w", WAVELETS)
def test_impulse_response_equals_closed_form_taps(w):
    h, g = fb.cdf_filters(w)
    n = 64
    # low-band output i sees x[2i + k] through h[k]; probe with impulses
    i = 12
    low = np.zeros(h.size)
    for t, k in enumerate(range(-(h.size // 2), h.size // 2 + 1)):
        x = np.zeros(n); x[2 * i + k] = 1.0
        low[t] = oracle.forward_1d(x, w)[i]
    assert np.max(np.abs(low - h)) < 1e-14
    high = np.zeros(g.size)
    for t, k in enumerate(range(-(g.size // 2), g.size // 2 + 1)):
        x = np.zeros(n); x[2 * i + 1 + k] = 1.0
        high[t] = oracle.forward_1d(x, w)[n // 2 + i]
    assert np.max(np.abs(high - g)) < 1e-14


@pytest.mark.parametrize("w", WAVELETS)
@pytest.mark.parametrize("n", [2, 4, 6, 8, 10, 12, 14, 16, 34])
def test_1d_matches_filter_bank_with_symmetric_extension(w, n):
    x = np.random.default_rng(n).standard_normal(n) * 100
    assert np.max(np.abs(oracle.forward_1d(x, w) - fb.analysis_1d(x, w))) < 1e-12


# ---- 2-D oracle vs direct 2-D filter bank -------------------------------------

@pytest.mark.parametrize("w", WAVELETS)
def test_2d_matches_filter_bank_all_small_even_sizes(w):
    rng = np.random.default_rng(7)
    for H in range(2, 17, 2):
        for W in range(2, 17, 2):
            x = rng.integers(0, 256, (H, W)).astype(np.float64)
            err = np.max(np.abs(oracle.forward(x, w, 1) - fb.analysis_2d(x, w, 1)))
            assert err < 1e-10, (H, W, err)


@pytest.mark.parametrize("w", WAVELETS)
@pytest.mark.parametrize("shape,levels", [((32, 48), 3), ((64, 64), 5),
                                          ((8, 16), 3), ((40, 24), 3)])
def test_multilevel_is_recursion_of_filter_bank(w, shape, levels):
    x = np.random.default_rng(1).integers(0, 256, shape).astype(np.float64)
    err = np.max(np.abs(oracle.forward(x, w, levels) - fb.analysis_2d(x, w, levels)))
    assert err < 1e-10


def test_mallat_layout_places_horizontal_detail_top_right():
    # a pattern varying only along columns (horizontal axis) has no vertical
    # detail: energy must appear in HL (top-right) only, besides LL
    H, W = 16, 16
    x = np.tile(((-1.0) ** np.arange(W)) * 10, (H, 1))
    c = oracle.forward(x, "cdf53", 1)
    ll, hl, lh, hh = oracle.subbands(c, 1, 1)
    assert np.max(np.abs(hl)) > 1
    assert np.max(np.abs(lh)) < 1e-12 and np.max(np.abs(hh)) < 1e-12


# ---- invariants ---------------------------------------------------------------

@pytest.mark.parametrize("w", WAVELETS)
@pytest.mark.parametrize("shape,levels", [((2, 2), 1), ((64, 48), 4),
                                          ((128, 128), 6), ((4, 256), 2)])
def test_perfect_reconstruction(w, shape, levels):
    x = np.random.default_rng(2).integers(0, 256, shape).astype(np.float64)
    r = oracle.inverse(oracle.forward(x, w, levels), w, levels)
    assert np.max(np.abs(r - x)) <= 1e-10 * np.max(np.abs(x))


@pytest.mark.parametrize("w", WAVELETS)
def test_inverse_of_arbitrary_coefficients_round_trips(w):
    c = np.random.default_rng(3).standard_normal((32, 32))
    assert np.max(np.abs(oracle.forward(oracle.inverse(c, w, 3), w, 3) - c)) < 1e-10


@pytest.mark.parametrize("w", WAVELETS)
@pytest.mark.parametrize("levels", [1, 3, 5])
def test_constant_image(w, levels):
    # the lifting constants carry ~15 significant digits, so exact zeros and
    # exact gain 1 hold to about 1e-15 relative per step
    x = np.full((64, 96), 77.0)
    tol = 1e-13 * 77.0 * 2 * levels
    c = oracle.forward(x, w, levels)
    for j in range(1, levels + 1):
        ll, hl, lh, hh = oracle.subbands(c, j, levels)
        assert np.max(np.abs(hl)) < tol
        assert np.max(np.abs(lh)) < tol
        assert np.max(np.abs(hh)) < tol
    ll, *_ = oracle.subbands(c, levels, levels)
    assert np.max(np.abs(ll - 77.0)) < tol


@pytest.mark.parametrize("w,deg_ok,margin", [("cdf53", 1, 1), ("cdf97", 3, 2)])
def test_vanishing_moments_interior(w, deg_ok, margin):
    """High bands vanish on polynomials up to the moment order, away from the
    mirror kinks (margin in quads at each edge); one degree more does not."""
    H, W = 48, 64
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    xs, ys = xx / W, yy / H
    for deg in range(deg_ok + 2):
        x = 100 * (xs ** deg + 0.5 * ys ** deg + 0.25 * (xs * ys) ** (deg // 2))
        c = oracle.forward(x, w, 1)
        _, hl, lh, hh = oracle.subbands(c, 1, 1)
        inner = (slice(margin, H // 2 - margin), slice(margin, W // 2 - margin))
        worst = max(np.max(np.abs(b[inner])) for b in (hl, lh, hh))
        if deg <= deg_ok:
            assert worst < 1e-9, (deg, worst)
        else:
            assert worst > 1e-6, (deg, worst)


@pytest.mark.parametrize("w", WAVELETS)
def test_linearity(w):
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal((2, 32, 32))
    lhs = oracle.forward(2.5 * x - 3.0 * y, w, 3)
    rhs = 2.5 * oracle.forward(x, w, 3) - 3.0 * oracle.forward(y, w, 3)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_multithreaded_equals_single_threaded():
    x = np.random.default_rng(5).integers(0, 256, (256, 192)).astype(np.float64)
    a = oracle.forward(x, "cdf97", 4, nthreads=1)
    b = oracle.forward(x, "cdf97", 4, nthreads=4)
    assert np.array_equal(a, b)
    assert np.array_equal(oracle.inverse(a, "cdf97", 4, 1),
                          oracle.inverse(a, "cdf97", 4, 4))


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((6, 8)), "cdf97", 2)     # 6 not divisible by 4
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((8, 8)), 7, 1)           # unknown wavelet


# ---- the non-separable scheme (Sec. 3) ------------------------------------------

def test_step_matrices_identities():
    """T_P = T_P^V T_P^H, S_U = S_U^V S_U^H, H and V commute, the inverse step
    is the step with the negated filter, and the constant split factors T_P
    into the separable P0 steps after the spatial P1 step."""
    rng = np.random.default_rng(6)
    for _ in range(20):
        zm, zn = np.exp(1j * rng.uniform(0, 2 * np.pi, 2))
        p, u = rng.standard_normal(2)
        M = nsm.step_matrices(p, u, zm, zn)
        assert np.allclose(M["TP"], M["TPV"] @ M["TPH"])
        assert np.allclose(M["TP"], M["TPH"] @ M["TPV"])
        assert np.allclose(M["SU"], M["SUV"] @ M["SUH"])
        assert np.allclose(M["SU"], M["SUH"] @ M["SUV"])
        N = nsm.step_matrices(-p, -u, zm, zn)
        assert np.allclose(N["TP"] @ M["TP"], np.eye(4))
        assert np.allclose(N["SU"] @ M["SU"], np.eye(4))
        # split: P = p + p z  ->  T_P = (T^V_{P0} T^H_{P0}) T_{P1}
        I = np.eye(4, dtype=complex)
        def tp(P, Ps):
            T = I.copy(); T[1, 0] = P; T[2, 0] = Ps; T[3, 0] = P * Ps
            T[3, 1] = Ps; T[3, 2] = P
            return T
        def su(U, Us):
            S = I.copy(); S[0, 1] = U; S[0, 2] = Us; S[0, 3] = U * Us
            S[1, 3] = Us; S[2, 3] = U
            return S
        T0 = nsm.step_matrices(p, u, zm, zn)
        sepP0 = I.copy(); sepP0[1, 0] = p; sepP0[3, 2] = p
        vP0 = I.copy(); vP0[2, 0] = p; vP0[3, 1] = p
        assert np.allclose(T0["TP"], vP0 @ sepP0 @ tp(p * zm, p * zn))
        sU0h = I.copy(); sU0h[0, 1] = u; sU0h[2, 3] = u
        sU0v = I.copy(); sU0v[0, 2] = u; sU0v[1, 3] = u
        assert np.allclose(T0["SU"], sU0v @ sU0h @ su(u / zm, u / zn))


@pytest.mark.parametrize("scheme", nsm.SCHEMES)
def test_model_steps_match_matrices_in_z_domain(scheme):
    """With periodic boundaries the model's steps are diagonalised by the 2-D
    DFT; each frequency must see exactly the paper's 4x4 step matrix."""
    rng = np.random.default_rng(8)
    ny, nx = 8, 16
    p, u = 0.7, -0.3
    q = [rng.standard_normal((ny, nx)) for _ in range(4)]
    ops = nsm.OpCounter()
    steps = nsm._pair_steps(scheme)
    out = q
    for kind, fn in steps:
        out = fn(out, p if kind == "P" else u, ops, "periodic")
    Q = np.stack([np.fft.fft2(t) for t in q])        # (4, ny, nx)
    O = np.stack([np.fft.fft2(t) for t in out])
    for kn in range(ny):
        for km in range(nx):
            zm = np.exp(2j * np.pi * km / nx)
            zn = np.exp(2j * np.pi * kn / ny)
            M = nsm.step_matrices(p, u, zm, zn)
            pair = M["SU"] @ M["TP"]
            assert np.allclose(O[:, kn, km], pair @ Q[:, kn, km], atol=1e-9)


@pytest.mark.parametrize("w", WAVELETS)
@pytest.mark.parametrize("scheme", nsm.SCHEMES)
@pytest.mark.parametrize("shape,levels", [((2, 2), 1), ((16, 24), 2), ((64, 64), 4)])
def test_separable_equals_nonseparable_fp64(w, scheme, shape, levels):
    x = np.random.default_rng(9).integers(0, 256, shape).astype(np.float64)
    ref = oracle.forward(x, w, levels)
    c = nsm.forward(x, w, levels, scheme)
    assert np.max(np.abs(c - ref)) <= 1e-12 * 255
    r = nsm.inverse(c, w, levels, scheme)
    assert np.max(np.abs(r - x)) <= 1e-11 * 255


def test_table1_steps_and_operations():
    gold = json.load(open(os.path.join(GOLDEN, "table1_steps_ops.json")))
    for w in WAVELETS:
        for scheme, key in (("separable", "separable_lifting"),
                            ("nonseparable", "nonseparable_lifting")):
            ops = nsm.OpCounter()
            nsm.forward_level(np.zeros((8, 8)), w, scheme, ops)
            assert ops.steps == gold[w][key]["steps"]
            assert ops.macs == gold[w][key]["ops"]


_ORIG_PREDICT = nsm.nonsep_predict_split
_ORIG_UPDATE = nsm.nonsep_update_split


def _mutant_predict(q, p, ops, bnd):
    """The split predict with the diagonal P1 P1* term dropped."""
    a, b, c, d = _ORIG_PREDICT(q, p, ops, bnd)
    return [a, b, c, d - p * p * nsm._shift(q[0], 1, 1, bnd)]


def _mutant_update(q, u, ops, bnd):
    """The split update reading the right instead of the left neighbour of b."""
    a, b, c, d = q
    wrong = nsm._shift(b, 1, 0, bnd) - nsm._shift(b, -1, 0, bnd)
    na, nb, nc, nd = _ORIG_UPDATE(q, u, ops, bnd)
    return [na + u * wrong, nb, nc, nd]


@pytest.mark.parametrize("mutant", [_mutant_predict, _mutant_update])
def test_planted_model_mistakes_are_caught(monkeypatch, mutant):
    """A dropped term or a wrong neighbour in the non-separable model must
    break its agreement with the separable oracle."""
    name = "nonsep_predict_split" if mutant is _mutant_predict else "nonsep_update_split"
    monkeypatch.setattr(nsm, name, mutant)
    x = np.random.default_rng(10).integers(0, 256, (16, 16)).astype(np.float64)
    c = nsm.forward(x, "cdf97", 1, "nonseparable")
    assert np.max(np.abs(c - oracle.forward(x, "cdf97", 1))) > 1e-3
