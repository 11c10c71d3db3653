"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: the pair set is checked by an
independent all-pairs x 27-image enumeration, the spline interior by solving its
matching conditions, Plummer by differentiating the paper's potential, and the
rest by closed forms, symmetry invariants and hand-worked values.
"""
import os

import numpy as np
import pytest

from oracle import SPLINE, PLUMMER
from oracle.brute import brute_forces, spline_coefficients

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid_positions(rng, n, box=1.0, bits=20):
    """Random positions on a dyadic grid (exact in FP32 and under whole-cell shifts)."""
    q = rng.integers(0, 2 ** bits, size=(n, 3))
    return (q.astype(np.float64) * (box / 2 ** bits)).astype(np.float32)


CASES = []
for n, K in [(2, 5), (3, 5), (64, 5), (64, 6), (500, 6), (500, 8), (2000, 8)]:
    for kind in (SPLINE, PLUMMER):
        CASES.append((n, K, kind))


@pytest.mark.parametrize("n,K,kind", CASES)
def test_oracle_matches_brute_force_random(orc, n, K, kind):
    rng = np.random.default_rng(n * 31 + K)
    pos = rng.random((n, 3)).astype(np.float32)
    eps = 0.3 / K
    a, pairs = orc.forces(pos, 1.0, K, 2, eps, kind, 1.0 / n, return_pairs=True)
    b, kept = brute_forces(pos, 1.0, K, 2, eps, kind, 1.0 / n)
    assert pairs == kept == orc.count_pairs(pos, 1.0, K, 2)
    scale = np.abs(b).max()
    assert np.abs(a - b).max() <= 1e-12 * scale


@pytest.mark.parametrize("K", [5, 6, 8])
def test_oracle_matches_brute_force_edges(orc, K):
    """Faces, box edges (x=0 and x just below L), coincident particles, a box of side != 1."""
    box = 2.5
    w = box / K
    rng = np.random.default_rng(K)
    pts = []
    for k in range(K):                       # exactly on cell faces
        pts.append([k * w, (k * 7 % K) * w, 0.0])
    pts += [[np.nextafter(np.float32(box), np.float32(0)), 0.1, 0.2],   # just below L
            [0.0, 0.0, 0.0],
            [0.0, 0.0, 0.0],                                           # coincident with the previous
            [box - 0.01 * w, box - 0.01 * w, box - 0.01 * w],           # straddles the corner with (0,0,0)
            [0.01 * w, 0.5 * w, box - 0.3 * w]]
    pts = np.array(pts, dtype=np.float64)
    pts = np.concatenate([pts, rng.random((200, 3)) * box]).astype(np.float32)
    eps = 0.4 * w
    for kind in (SPLINE, PLUMMER):
        a, pairs = orc.forces(pts, box, K, 2, eps, kind, 0.01, return_pairs=True)
        b, kept = brute_forces(pts, box, K, 2, eps, kind, 0.01)
        assert pairs == kept
        assert np.all(np.isfinite(a))
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_oracle_positions_outside_box_are_wrapped(orc):
    rng = np.random.default_rng(5)
    pos = rng.random((300, 3)).astype(np.float32)
    shifted = pos.astype(np.float64)
    shifted[:100] += 1.0
    shifted[100:200] -= 2.0
    shifted = shifted.astype(np.float32)
    keep = np.all((shifted.astype(np.float64) - np.floor(shifted.astype(np.float64))) == pos.astype(np.float64), axis=1)
    a = orc.forces(pos[keep], 1.0, 6, 2, 0.05, SPLINE, 1.0)
    b = orc.forces(shifted[keep], 1.0, 6, 2, 0.05, SPLINE, 1.0)
    assert np.array_equal(a, b)


def test_golden_two_body_values(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "two_body.txt")) if l.strip() and not l.startswith("#")]
    for kind, eps, r, f in rows:
        kind, eps, r, f = int(kind), float(eps), float(r), float(f)
        g = orc.kernel_g(np.array([r]), eps, kind)[0]
        assert g * r == pytest.approx(f, rel=1e-14, abs=0.0)


@pytest.mark.parametrize("kind", [SPLINE, PLUMMER])
def test_two_body_in_a_box(orc, kind):
    """Two particles, one pair: equal and opposite forces along the separation."""
    eps = 0.05
    for sep in (0.01, 0.03, 0.049, 0.05, 0.07, 0.2):
        pos = np.array([[0.5, 0.5, 0.5], [0.5 + sep, 0.5, 0.5]], dtype=np.float32)
        r = float(np.float64(pos[1, 0]) - np.float64(pos[0, 0]))
        a = orc.forces(pos, 1.0, 5, 2, eps, kind, 0.7)
        mag = 0.7 * orc.kernel_g(np.array([r]), eps, kind)[0] * r
        assert a[0, 0] == pytest.approx(mag, rel=1e-14) and a[0, 0] > 0
        assert a[1, 0] == pytest.approx(-mag, rel=1e-14)
        assert a[0, 1] == a[0, 2] == a[1, 1] == a[1, 2] == 0.0


def test_spline_is_newtonian_beyond_eps(orc):
    eps = 0.013
    r = np.concatenate([[eps], eps * (1 + np.geomspace(1e-12, 100, 500))])
    g = orc.kernel_g(r, eps, SPLINE)
    np.testing.assert_allclose(g * r ** 3, 1.0, rtol=2e-15, atol=0)


def test_spline_interior_matches_c2_conditions(orc):
    """The interior force equals the cubic whose value, slope and curvature match 1/r^2 at eps
    (coefficients solved numerically here, not typed)."""
    for eps in (0.5, 0.013, 3e-4):
        a, b, c = spline_coefficients(eps)
        r = np.linspace(0, eps, 1001)[1:-1]
        f = orc.kernel_g(r, eps, SPLINE) * r
        np.testing.assert_allclose(f, a * r + b * r ** 2 + c * r ** 3, rtol=1e-12)


def test_spline_continuity_at_eps(orc):
    """C0, C1 and C2 continuity of the force at r = eps, by one-sided differences."""
    eps = 1.0
    F = lambda r: orc.kernel_g(np.atleast_1d(r), eps, SPLINE) * np.atleast_1d(r)
    h = 1e-4
    left = F(np.array([eps - 2 * h, eps - h, eps]))
    right = F(np.array([eps, eps + h, eps + 2 * h]))
    assert left[2] == pytest.approx(1.0, rel=1e-15)
    d1l = (3 * left[2] - 4 * left[1] + left[0]) / (2 * h)
    d1r = (-3 * right[0] + 4 * right[1] - right[2]) / (2 * h)
    assert d1l == pytest.approx(-2.0, rel=1e-6) and d1r == pytest.approx(-2.0, rel=1e-6)
    d2l = (left[2] - 2 * left[1] + left[0]) / h ** 2
    d2r = (right[0] - 2 * right[1] + right[2]) / h ** 2
    assert d2l == pytest.approx(6.0, rel=1e-3) and d2r == pytest.approx(6.0, rel=1e-3)
    # the core is finite: g(0+) = 10/eps^3 and the force vanishes at r -> 0
    assert orc.kernel_g(np.array([1e-12]), eps, SPLINE)[0] == pytest.approx(10.0, rel=1e-10)


def test_plummer_is_the_gradient_of_its_potential(orc):
    """Force magnitude = -dphi/dr of phi = -1/sqrt(r^2+eps^2), by Richardson-extrapolated differences."""
    eps = 0.2
    phi = lambda r: -1.0 / np.sqrt(r * r + eps * eps)
    r = np.linspace(0.01, 1.0, 200)
    def d(h):
        return (phi(r + h) - phi(r - h)) / (2 * h)
    dphi = (4 * d(1e-4) - d(2e-4)) / 3
    f = orc.kernel_g(r, eps, PLUMMER) * r
    np.testing.assert_allclose(f, dphi, rtol=1e-8)


def test_spline_is_the_gradient_of_its_potential(orc):
    """Integrate the spline force numerically from r to far away: potential -> -1/r outside eps,
    and the interior potential is finite (a softened core)."""
    eps = 1.0
    r = np.linspace(1e-6, 3.0, 300001)
    f = orc.kernel_g(r, eps, SPLINE) * r
    # potential phi(r) = -int_r^inf F; beyond 3 it is -1/r exactly
    seg = np.concatenate([[0.0], np.cumsum((f[1:] + f[:-1]) * 0.5 * np.diff(r))])
    phi = -(seg[-1] - seg) - 1.0 / 3.0
    out = r >= 1.0
    np.testing.assert_allclose(phi[out], -1.0 / r[out], rtol=1e-8, atol=1e-9)
    assert np.isfinite(phi[0]) and phi[0] < -1.0


@pytest.mark.parametrize("K,off", [(5, (0.5, 0.5, 0.5)), (6, (0.125, 0.75, 0.3125)), (8, (0.0, 0.25, 0.875))])
def test_lattice_has_zero_force(orc, K, off):
    """One particle per cell at a common offset: the 5^3 block is symmetric, so every force is 0.
    Cell width 1/2 and dyadic offsets keep the lattice exact in FP32."""
    w = 0.5
    box = K * w
    g = np.stack(np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij"), -1).reshape(-1, 3)
    pos = ((g + np.array(off)) * w).astype(np.float32)
    assert np.array_equal(pos.astype(np.float64), (g + np.array(off)) * w)
    gm = 1.0 / len(pos)
    for kind in (SPLINE, PLUMMER):
        a = orc.forces(pos, box, K, 2, 0.3 * w, kind, gm)
        assert np.abs(a).max() <= 1e-13 * gm / w ** 2


def test_lattice_two_per_cell_is_not_zero(orc):
    """Guard for the previous pin: with two particles per cell the block is asymmetric."""
    K, w = 6, 1.0 / 6
    g = np.stack(np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij"), -1).reshape(-1, 3)
    pos = np.concatenate([(g + 0.3) * w, (g + 0.6) * w]).astype(np.float32)
    a = orc.forces(pos, 1.0, K, 2, 0.01, SPLINE, 1.0)
    assert np.abs(a).max() > 1.0


@pytest.mark.parametrize("kind", [SPLINE, PLUMMER])
def test_momentum_conservation(orc, kind):
    """Newton's third law: the pair set is symmetric and the pair force antisymmetric, so sum a_i = 0."""
    rng = np.random.default_rng(11)
    n, K = 3000, 7
    pos = np.concatenate([rng.random((2000, 3)), 0.5 + 0.02 * rng.standard_normal((1000, 3))]).astype(np.float32) % 1
    a = orc.forces(pos, 1.0, K, 2, 0.01, kind, 1.0 / n)
    assert np.linalg.norm(a.sum(axis=0)) <= 1e-12 * np.linalg.norm(a, axis=1).sum()


def test_translation_by_whole_cells(orc):
    rng = np.random.default_rng(3)
    K = 8
    pos = _grid_positions(rng, 1500)
    a = orc.forces(pos, 1.0, K, 2, 0.02, SPLINE, 1.0)
    shift = np.array([3, -2, 7]) / K
    moved = np.mod(pos.astype(np.float64) + shift, 1.0).astype(np.float32)
    b = orc.forces(moved, 1.0, K, 2, 0.02, SPLINE, 1.0)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


def test_permutation_invariance(orc):
    rng = np.random.default_rng(4)
    pos = rng.random((2500, 3)).astype(np.float32)
    a = orc.forces(pos, 1.0, 6, 2, 0.02, PLUMMER, 1.0)
    p = rng.permutation(len(pos))
    b = orc.forces(pos[p], 1.0, 6, 2, 0.02, PLUMMER, 1.0)
    np.testing.assert_allclose(b, a[p], rtol=1e-12, atol=1e-13 * np.abs(a).max())


def test_sink_subset_matches_full(orc):
    rng = np.random.default_rng(8)
    pos = rng.random((3000, 3)).astype(np.float32)
    full = orc.forces(pos, 1.0, 6, 2, 0.02, SPLINE, 1.0)
    sinks = np.array([0, 17, 2999, 1500, 17])
    sub = orc.forces(pos, 1.0, 6, 2, 0.02, SPLINE, 1.0, sinks=sinks)
    assert np.array_equal(sub, full[sinks])


def test_neumaier_agrees_with_plain(orc):
    rng = np.random.default_rng(9)
    pos = np.concatenate([rng.random((4000, 3)), 0.3 + 0.01 * rng.standard_normal((4000, 3))]).astype(np.float32) % 1
    a = orc.forces(pos, 1.0, 8, 2, 0.005, SPLINE, 1.0)
    b = orc.forces(pos, 1.0, 8, 2, 0.005, SPLINE, 1.0, neumaier=True)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_cell_rule_edges(orc):
    """Faces go to the upper cell; values that wrap or round to L go to the last cell."""
    K = 8
    below_one = float(np.nextafter(np.float32(1), np.float32(0)))
    pts = np.array([[0.0, 0.125, 0.25],          # exactly on faces -> cells 0, 1, 2
                    [0.124999993, 0.5, 0.875],   # just below a face -> 0; faces -> 4, 7
                    [below_one, 0.0, 0.999],     # -> 7, 0, 7
                    [-1e-30, 1.0, 2.0625],       # wraps: -> 7 (rounds to L), 0, 0
                    [-0.125, 1.125, -3.0]],      # -> 7, 1, 0
                   dtype=np.float32)
    want = np.array([[0, 1, 2], [0, 4, 7], [7, 0, 7], [7, 0, 0], [7, 1, 0]])
    lin = (want[:, 0] * K + want[:, 1]) * K + want[:, 2]
    assert np.array_equal(orc.bin_cells(pts, 1.0, K), lin)


def test_empty_and_invalid_arguments(orc):
    assert orc.forces(np.zeros((0, 3), np.float32), 1.0, 5, 2, 0.1).shape == (0, 3)
    with pytest.raises(ValueError):
        orc.forces(np.zeros((4, 3), np.float32), 1.0, 4, 2, 0.1)     # K < 2R+1
    with pytest.raises(ValueError):
        orc.forces(np.zeros((4, 3), np.float32), 1.0, 5, 2, 0.0)     # eps <= 0


# ---------------------------------------------------------------- kernel density estimate (Sec. 3.3)

@pytest.mark.parametrize("n,K", [(2, 5), (300, 5), (2000, 7)])
def test_density_matches_brute_force(orc, n, K):
    from oracle.brute import brute_density
    rng = np.random.default_rng(n + K)
    pos = rng.random((n, 3)).astype(np.float32)
    pos[:2] = [[0.001, 0.5, 0.5], [0.999, 0.5, 0.5]]     # a pair across the periodic boundary
    b = 0.6 / K
    rho = orc.density(pos, 1.0, K, 2, b)
    ref = brute_density(pos, 1.0, K, 2, b)
    assert np.abs(rho - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_density_closed_forms(orc):
    # isolated particles: only the self pair, weight 1
    pos = np.array([[0.1, 0.1, 0.1], [0.6, 0.6, 0.6]], np.float32)
    assert np.array_equal(orc.density(pos, 1.0, 5, 2, 0.05), [1.0, 1.0])
    # a pair at distance r < b: 1 + (1 - r^2/b^2) each; r = b/2 -> 1.75
    pos = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5625]], np.float32)
    np.testing.assert_allclose(orc.density(pos, 1.0, 5, 2, 0.125), [1.75, 1.75], rtol=1e-15)
    # exactly at r = b the weight vanishes
    np.testing.assert_allclose(orc.density(pos, 1.0, 5, 2, 0.0625), [1.0, 1.0], rtol=1e-15)


def test_density_lattice(orc):
    """Simple cubic lattice of spacing a: with a < b < sqrt(2) a each particle sees itself and its
    6 face neighbours at distance a: rho = 1 + 6 (1 - a^2/b^2)."""
    K, per = 6, 2
    m = K * per
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    a = 0.5                                   # dyadic spacing: the lattice is exact in FP32
    pos = ((g + 0.5) * a).astype(np.float32)
    b = 1.25 * a
    rho = orc.density(pos, m * a, K, 2, b)
    np.testing.assert_allclose(rho, 1 + 6 * (1 - 1 / 1.25 ** 2), rtol=1e-12)


# ---------------------------------------------------------------- cell multipoles (Sec. 3.1, order 8)

def test_multipole_component_order_and_count():
    from oracle import multipole_exponents
    e = multipole_exponents(8)
    assert len(e) == 165 == len(set(e))
    assert e[0] == (0, 0, 0) and e[1:4] == [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    assert all(sum(t) <= 8 for t in e)


def test_multipoles_single_particle_closed_form(orc):
    """One particle at cell-relative (u, v, w): every moment is m u^a v^b w^k (dyadic values, exact)."""
    from oracle import multipole_exponents
    K, L = 4, 1.0
    u, v, w = 0.25, -0.375, 0.125
    cell = (2, 1, 3)
    pos = np.array([[(cell[0] + 0.5 + u) / K, (cell[1] + 0.5 + v) / K, (cell[2] + 0.5 + w) / K]], np.float32)
    M = orc.multipoles(pos, L, K, 8, 2.0)
    lin = (cell[0] * K + cell[1]) * K + cell[2]
    want = np.array([2.0 * u ** a * v ** b * w ** k for a, b, k in multipole_exponents(8)])
    assert np.array_equal(M[lin], want)
    assert np.count_nonzero(np.delete(M, lin, axis=0)) == 0


def test_multipoles_symmetric_pairs_cancel_odd_orders(orc):
    """Pairs mirrored through the cell centre: all odd-degree moments vanish, even ones double."""
    from oracle import multipole_exponents
    K = 4                                                                  # dyadic cell width: exact positions
    rng = np.random.default_rng(2)
    off = (rng.integers(-2 ** 10, 2 ** 10, size=(50, 3)) / 2 ** 12)        # dyadic offsets, |off| < 1/4
    centre = np.array([1.5, 1.5, 1.5])
    pos = np.concatenate([centre + off, centre - off]) / K
    M = orc.multipoles(pos.astype(np.float32), 1.0, K, 8, 1.0)
    mid = (1 * K + 1) * K + 1
    for (a, b, k), val in zip(multipole_exponents(8), M[mid]):
        if (a + b + k) % 2:
            assert abs(val) <= 1e-15
        else:
            assert val == pytest.approx(2 * np.sum(off[:, 0] ** a * off[:, 1] ** b * off[:, 2] ** k), rel=1e-12)


def test_multipoles_monopole_and_dipole_are_mass_and_centre_of_mass(orc):
    rng = np.random.default_rng(3)
    K = 5
    pos = rng.random((4000, 3)).astype(np.float32)
    m = 0.37
    M = orc.multipoles(pos, 1.0, K, 2, m)
    c = np.minimum(np.floor(pos.astype(np.float64) * K), K - 1).astype(np.int64)
    lin = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    counts = np.bincount(lin, minlength=K ** 3)
    assert np.allclose(M[:, 0], m * counts, rtol=0, atol=1e-12)
    rel = pos.astype(np.float64) * K - (c + 0.5)
    for d in range(3):
        assert np.allclose(M[:, 1 + d], m * np.bincount(lin, weights=rel[:, d], minlength=K ** 3), atol=1e-11)


def test_multipoles_shift_theorem(orc):
    """Moments about a displaced centre follow from the cell moments by the binomial theorem:
    sum_j (u_j + h)^a = sum_i C(a, i) h^(a-i) M^(i).  Checked for the x-exponent of every component."""
    from math import comb
    from oracle import multipole_exponents
    rng = np.random.default_rng(4)
    K = 2
    pos = (rng.random((300, 3)) * 0.5).astype(np.float32)        # all in cell (0, 0, 0)
    M = orc.multipoles(pos, 1.0, K, 8, 1.0)[0]
    idx = {e: i for i, e in enumerate(multipole_exponents(8))}
    rel = pos.astype(np.float64) * K - 0.5
    h = 0.3
    for (a, b, k) in multipole_exponents(8):
        direct = np.sum((rel[:, 0] + h) ** a * rel[:, 1] ** b * rel[:, 2] ** k)
        shifted = sum(comb(a, i) * h ** (a - i) * M[idx[(i, b, k)]] for i in range(a + 1))
        assert shifted == pytest.approx(direct, rel=1e-10, abs=1e-12)


# ---------------------------------------------------------------- far field from cell Taylor series (Sec. 3.1)

def test_taylor_linear_and_quadratic_potentials(orc):
    """Phi = g u gives a_x = -(K/L) g everywhere; Phi = h v^2 gives a_y = -(K/L) 2 h v (dyadic inputs, exact)."""
    from oracle import multipole_exponents
    K, L, p = 4, 2.0, 8
    e = multipole_exponents(p)
    T = np.zeros((K ** 3, len(e)))
    T[:, e.index((1, 0, 0))] = 3.0
    T[:, e.index((0, 2, 0))] = -0.5
    rng = np.random.default_rng(1)
    pos = (rng.integers(0, 2 ** 12, size=(500, 3)) / 2 ** 12 * L).astype(np.float32)
    a = orc.taylor_forces(pos, L, K, p, T)
    x = pos.astype(np.float64) * (K / L)
    v = x[:, 1] - (np.minimum(np.floor(x[:, 1]), K - 1) + 0.5)
    assert np.all(a[:, 0] == -(K / L) * 3.0)
    assert np.allclose(a[:, 1], (K / L) * 2 * 0.5 * v, rtol=0, atol=1e-15)
    assert np.all(a[:, 2] == 0.0)
    acc0 = rng.random((500, 3))
    assert np.allclose(orc.taylor_forces(pos, L, K, p, T, acc0), acc0 + a, rtol=0, atol=1e-14)   # co-add


def test_taylor_series_of_a_distant_mass_reproduces_its_force(orc):
    """Fit the order-8 Taylor polynomial of Phi = -1/|x - x0| about one cell centre from samples (a plain
    least-squares fit, independent of the oracle), then the oracle's gradient must match the exact force of
    the distant mass to the truncation error of the series."""
    from oracle import multipole_exponents
    K, L, p = 8, 1.0, 8
    w = L / K
    cell = np.array([3, 4, 2])
    centre = (cell + 0.5) * w
    x0 = centre + np.array([0.41, -0.27, 0.33])              # ~4 cell widths away
    e = multipole_exponents(p)
    rng = np.random.default_rng(7)
    u = rng.uniform(-0.5, 0.5, size=(4000, 3))
    phi = -1.0 / np.linalg.norm(centre + u * w - x0, axis=1)
    A = np.stack([u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** k for a, b, k in e], axis=1)
    coef = np.linalg.lstsq(A, phi, rcond=None)[0]
    T = np.zeros((K ** 3, len(e)))
    T[(cell[0] * K + cell[1]) * K + cell[2]] = coef
    pts = centre + rng.uniform(-0.45, 0.45, size=(200, 3)) * w
    acc = orc.taylor_forces(pts.astype(np.float32), L, K, p, T)
    d = x0 - pts.astype(np.float32).astype(np.float64)
    exact = d / np.linalg.norm(d, axis=1)[:, None] ** 3       # -grad(-1/r) points to the mass
    assert np.allclose(acc, exact, rtol=1e-6, atol=1e-6 * np.abs(exact).max())
