"""The column arithmetic of the kernels' edge loads, checked exhaustively on
the CPU: a lane that reads E consecutive elements at an E-aligned start
loads two aligned E-element vectors at `base` and base + E, where base is the
smallest mirrored column rounded down to a multiple of E, and selects its
elements from them. For rows whose length is a multiple of E this must
(1) cover every mirrored column the lane stands for, (2) keep the first
vector inside the row and (3) leave the second either wholly inside or
wholly outside it, so that no vector load is partly out of range. The same
holds for the inverse's per-phase quad indices."""
import pytest


def mirror(x, n):
    """Whole-sample symmetric extension of an n-sample axis (period 2n-2)."""
    if x < 0:
        x = -x
    if x < n:
        return x
    p = 2 * n - 2
    if x >= p:
        x %= p
    return x if x < n else p - x


def _check(m, x0, n, E, plain):
    base = x0 if plain else (min(m) & ~(E - 1))
    assert all(0 <= v < n for v in m)
    assert all(base <= v < base + 2 * E for v in m)
    assert base >= 0 and base + E <= n
    assert base + 2 * E <= n or base + E >= n
    if plain:
        assert m == list(range(x0, x0 + E))


def test_mirror_matches_the_periodic_definition():
    for n in range(2, 30):
        period = 2 * n - 2
        for x in range(-100, 100):
            r = x % period
            assert mirror(x, n) == (r if r < n else period - r)


@pytest.mark.parametrize("E", [2, 4, 8])
def test_forward_columns(E):
    for n in range(E, 160, E):
        for x0 in range(-8 * E, n + 8 * E, E):
            m = [mirror(x0 + k, n) for k in range(E)]
            _check(m, x0, n, E, x0 >= 0 and x0 + E <= n)


@pytest.mark.parametrize("E", [1, 2, 4])
def test_inverse_phase_columns(E):
    for nq in range(E, 100, E):
        w = 2 * nq
        for q0 in range(-8 * E, nq + 8 * E, E):
            xe = [mirror(2 * (q0 + i), w) >> 1 for i in range(E)]
            xo = [(mirror(2 * (q0 + i) + 1, w) - 1) >> 1 for i in range(E)]
            plain = q0 >= 0 and q0 + E <= nq
            _check(xe, q0, nq, E, plain)
            _check(xo, q0, nq, E, plain)
