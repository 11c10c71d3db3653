"""The pins must catch plausible mistakes: each test plants one mistake in a
copy of the oracle source, builds it on the CPU, and checks that the pin
battery rejects it (and that the unmodified source passes the same battery)."""
import os

import numpy as np
import pytest

import oracle
from oracle import SPLINE, PLUMMER
from oracle.brute import brute_forces, spline_coefficients

MUTANTS = {
    "spline_coefficient": ("(10.0 - 15.0 * u + 6.0 * u * u)", "(10.0 - 14.0 * u + 6.0 * u * u)"),
    "spline_sign": ("(10.0 - 15.0 * u + 6.0 * u * u)", "(10.0 + 15.0 * u + 6.0 * u * u)"),
    "image_shift_sign": ("if (ex < 0) { ex += K; sx = -1; }", "if (ex < 0) { ex += K; sx = 1; }"),
    "dropped_dz_term": ("double r2 = ddx * ddx + ddy * ddy + ddz * ddz;", "double r2 = ddx * ddx + ddy * ddy;"),
    "transposed_operands": ("double ddy = (xt[3 * j + 1] + sy * L) - yi;", "double ddy = yi - (xt[3 * j + 1] + sy * L);"),
    "window_off_by_one": ("for (int dz = -R; dz <= R; dz++) {\n                    int ez", "for (int dz = -R; dz < R; dz++) {\n                    int ez"),
    "plummer_eps_power": ("double q = r2 + eps * eps;", "double q = r2 + eps;"),
    "cell_rule_round": ("double f = floor(t);", "double f = floor(t + 0.5);"),
    "cutover_radius": ("if (r >= eps) return 1.0 / (r2 * r);", "if (r >= 0.9 * eps) return 1.0 / (r2 * r);"),
    "mass_applied_twice": ("acc[3 * q + 1] = gm * (a.s1 + a.c1);", "acc[3 * q + 1] = gm * gm * (a.s1 + a.c1);"),
    "neighbour_x_wrap": ("else if (ex >= K) { ex -= K; sx = 1; }", "else if (ex >= K) { ex -= K; sx = 0; }"),
    "density_weight_power": ("double w = 1.0 - (ddx * ddx + ddy * ddy + ddz * ddz) / b2;",
                             "double w = 1.0 - sqrt(ddx * ddx + ddy * ddy + ddz * ddz) / b;"),
    "multipole_centre": ("t[d] = xt * s - ((double)c[d] + 0.5);", "t[d] = xt * s - (double)c[d];"),
    "multipole_power": ("pw[q] = pw[q - 1] * t[2];", "pw[q] = pw[q - 1] * t[1];"),
    "multipole_order": ("for (int b = deg - a; b >= 0; b--) {", "for (int b = 0; b <= deg - a; b++) {"),
    "taylor_sign": ("acc[3 * i + 1] -= s * gy;", "acc[3 * i + 1] += s * gy;"),
    "taylor_scale": ("acc[3 * i + 0] -= s * gx;", "acc[3 * i + 0] -= gx;"),
    "taylor_derivative": ("if (k > 0) gz += T[idx] * k * pw3[0][a] * pw3[1][b] * pw3[2][k - 1];",
                          "if (k > 0) gz += T[idx] * pw3[0][a] * pw3[1][b] * pw3[2][k - 1];"),
    "density_self_excluded": ("if (w > 0.0) sum += w;", "if (w > 0.0 && w < 1.0) sum += w;"),
    "density_image_dropped": ("double ddz = (xt[3 * j + 2] + sz * L) - zi;\n                        double w",
                              "double ddz = xt[3 * j + 2] - zi;\n                        double w"),
}


def battery(o: oracle.Oracle) -> list:
    """Run the core pins against one oracle build; return the names of those that fail."""
    bad = []
    rng = np.random.default_rng(0)
    for K in (5, 7):
        pos = rng.random((300, 3)).astype(np.float32)
        pos[:3] = [[0.0, 0.0, 0.0], [0.999, 0.999, 0.999], [0.0, 0.0, 0.0]]
        for kind in (SPLINE, PLUMMER):
            a = o.forces(pos, 1.0, K, 2, 0.2 / K, kind, 0.37)
            b, _ = brute_forces(pos, 1.0, K, 2, 0.2 / K, kind, 0.37)
            if not (np.all(np.isfinite(a)) and np.abs(a - b).max() <= 1e-12 * np.abs(b).max()):
                bad.append(f"brute K={K} kind={kind}")
    eps = 0.05
    ca, cb, cc = spline_coefficients(eps)
    r = np.linspace(0, eps, 101)[1:-1]
    if not np.allclose(o.kernel_g(r, eps, SPLINE) * r, ca * r + cb * r ** 2 + cc * r ** 3, rtol=1e-12):
        bad.append("spline c2")
    r = np.linspace(0.01, 1.0, 50)
    phi = lambda x: -1.0 / np.sqrt(x * x + 0.04)
    dphi = (phi(r + 1e-5) - phi(r - 1e-5)) / 2e-5
    if not np.allclose(o.kernel_g(r, 0.2, PLUMMER) * r, dphi, rtol=1e-6):
        bad.append("plummer gradient")
    pts = np.array([[0.0, 0.125, 0.25], [0.124999993, 0.5, 0.875]], dtype=np.float32)
    if not np.array_equal(o.bin_cells(pts, 1.0, 8), [(0 * 8 + 1) * 8 + 2, (0 * 8 + 4) * 8 + 7]):
        bad.append("cell rule")
    from oracle.brute import brute_density
    pos = rng.random((300, 3)).astype(np.float32)
    pos[:2] = [[0.5, 0.5, 0.001], [0.5, 0.5, 0.999]]
    if not np.allclose(o.density(pos, 1.0, 5, 2, 0.12), brute_density(pos, 1.0, 5, 2, 0.12), rtol=1e-12, atol=0):
        bad.append("density")
    from oracle import multipole_exponents
    q = np.array([[(2.5 + 0.25) / 4, (1.5 - 0.375) / 4, (0.5 + 0.125) / 4]], np.float32)
    M = o.multipoles(q, 1.0, 4, 8, 1.0)[(2 * 4 + 1) * 4 + 0]
    if not np.array_equal(M, [0.25 ** a * (-0.375) ** b * 0.125 ** k for a, b, k in multipole_exponents(8)]):
        bad.append("multipoles")
    e = multipole_exponents(8)
    T = np.zeros((4 ** 3, len(e)))
    T[:, e.index((1, 0, 0))] = 1.0
    T[:, e.index((0, 1, 0))] = 2.0
    T[:, e.index((0, 0, 3))] = 1.0
    pts = np.array([[0.3, 0.55, 0.8125]], np.float32)                  # w = (0.8125*4 - 3.5) = -0.25
    if not np.allclose(o.taylor_forces(pts, 1.0, 4, 8, T), [[-4.0, -8.0, -4.0 * 3 * 0.0625]], rtol=1e-12):
        bad.append("taylor")
    return bad


def _build_variant(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    if old is not None:
        assert src.count(old) >= 1, f"mutation anchor for {name} not found"
        src = src.replace(old, new, 1)   # the first occurrence: the force sum (the density follows it)
    path = os.path.join(tmp_path, f"oracle_{name}.c")
    open(path, "w").write(src)
    return oracle.Oracle(oracle.compile_oracle(path, os.path.join(tmp_path, f"liboracle_{name}.so")))


def test_unmodified_oracle_passes_battery(tmp_path):
    assert battery(_build_variant(str(tmp_path), "clean", None, None)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert battery(_build_variant(str(tmp_path), name, old, new)) != []
