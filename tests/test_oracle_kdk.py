"""Pins of the leapfrog / timestep oracle (oracle/kdk.py) against closed forms, invariants of the
integrator and planted mistakes (Sec. 2.5, time stepping, Sec. 3.1 kick / drift / rebin)."""
import os
import types

import numpy as np
import pytest

import oracle
from oracle import PLUMMER, SPLINE
from oracle import kdk as kdk_mod

KDK_SRC = os.path.join(os.path.dirname(oracle.__file__), "kdk.py")


# ---------------------------------------------------------------- the pins, as a battery over a module

def pin_kick_closed_form(m):
    v = np.array([[1.0, -2.0, 0.5]], np.float32)
    a = np.array([[2.0, 4.0, -8.0]], np.float32)
    return np.array_equal(m.kick(v, a, 0.25), np.array([[1.5, -1.0, -1.5]], np.float32))


def pin_drift_wraps(m):
    x = np.array([[0.75, 0.25, 0.5]], np.float32)
    v = np.array([[0.5, -0.5, 2.0]], np.float32)
    # 0.75 + 0.5 -> 1.25 -> 0.25; 0.25 - 0.5 -> -0.25 -> 0.75; 0.5 + 2 -> 2.5 -> 0.5 (two boxes)
    return np.array_equal(m.drift(x, v, 1.0, 1.0), np.array([[0.25, 0.75, 0.5]], np.float32))


def pin_drift_round_up_to_box_is_zero(m):
    # 1 - 2^-30 is below the box in FP64 but rounds to 1.0 in FP32: stored as 0
    x = np.array([[0.5, 0.5, 0.5]], np.float32)
    got = m.drift(x, np.array([[0.5, 0.0, 0.0]], np.float32), 1.0 - 2.0 ** -30, 1.0)
    return got[0, 0] == 0.0 and got[0, 1] == 0.5


def pin_free_streaming(m):
    """A lone particle feels no force: after n steps it has moved by v * sum(dt), wrapped."""
    x = np.array([[0.1, 0.2, 0.3]], np.float32)
    v = np.array([[0.25, -0.125, 0.0625]], np.float32)
    f = m.near_field(1.0, 5, 2, 0.01, SPLINE, 1.0)
    xs, vs, _ = m.kdk_steps(x, v, [0.5, 0.5, 1.0, 2.0], 1.0, f)
    want = (np.array([0.1, 0.2, 0.3]) + 4.0 * np.array([0.25, -0.125, 0.0625])) % 1.0
    return np.array_equal(vs, v) and np.allclose(xs[0], want, rtol=0, atol=3e-7)


def _oscillator_error(m, dt, t_end=2.0):
    """Isotropic harmonic oscillator about the box centre, a = -(x - 1/2); exact x(t) known."""
    x0 = np.array([[0.6, 0.45, 0.5]], np.float32)
    v0 = np.array([[0.0, 0.08, -0.05]], np.float32)
    f = lambda p: -(np.asarray(p, np.float64) - 0.5)
    n = int(round(t_end / dt))
    xs, vs, _ = m.kdk_steps(x0, v0, [dt] * n, 1.0, f)
    c = x0.astype(np.float64) - 0.5
    exact = 0.5 + c * np.cos(t_end) + v0.astype(np.float64) * np.sin(t_end)
    return float(np.abs(xs.astype(np.float64) - exact).max())


def pin_second_order(m):
    e1, e2, e3 = (_oscillator_error(m, dt) for dt in (0.2, 0.1, 0.05))
    return 3.5 < e1 / e2 < 4.5 and 3.5 < e2 / e3 < 4.5


def _random_system(n=200, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)).astype(np.float32)
    v = (0.05 * rng.standard_normal((n, 3))).astype(np.float32)
    return x, v


def pin_time_reversible(m):
    """Forward dt then backward -dt returns to the start up to FP32 storage rounding."""
    x, v = _random_system()
    f = m.near_field(1.0, 5, 2, 0.04, PLUMMER, 1.0 / 200)
    x1, v1, _ = m.kdk_step(x, v, 0.05, 1.0, f)
    x2, v2, _ = m.kdk_step(x1, v1, -0.05, 1.0, f)
    dx = np.abs(((x2.astype(np.float64) - x + 0.5) % 1.0) - 0.5)
    moved = np.abs(((x1.astype(np.float64) - x + 0.5) % 1.0) - 0.5).max()
    return moved > 1e-3 and dx.max() < 1e-6 and np.abs(v2.astype(np.float64) - v).max() < 1e-6


def pin_momentum_conserved(m):
    """Pairwise antisymmetric forces: the mean velocity does not change (to FP32 rounding)."""
    x, v = _random_system(seed=4)
    f = m.near_field(1.0, 5, 2, 0.04, SPLINE, 1.0 / 200)
    _, v1, _ = m.kdk_steps(x, v, [0.05, 0.05], 1.0, f)
    dv = np.abs(v1.astype(np.float64) - v).max()
    return dv > 1e-3 and np.abs(v1.astype(np.float64).sum(0) - v.astype(np.float64).sum(0)).max() < 1e-5


def pin_timestep_closed_form(m):
    """K=2: cell 0 holds two particles with velocities +-u along x and accelerations of norm 3 and 5
    (sigma = u, max|a| = 5); cell 7 holds three with velocities (w, 0, 0), (-w, 0, 0), (0, 0, 0) and
    |a| = 1 (sigma = w sqrt(2/3)); cell 1 holds one (ignored)."""
    u, w = 0.3, 0.2
    pos = np.array([[0.1, 0.1, 0.1], [0.2, 0.2, 0.2], [0.7, 0.7, 0.7], [0.8, 0.8, 0.8], [0.9, 0.6, 0.7],
                    [0.1, 0.1, 0.9]], np.float32)
    vel = np.array([[u, 0, 0], [-u, 0, 0], [w, 0, 0], [-w, 0, 0], [0, 0, 0], [9, 9, 9]], np.float32)
    acc = np.array([[3, 0, 0], [0, 4, 3], [0, 1, 0], [1, 0, 0], [0, 0, 1], [1e-3, 0, 0]], np.float32)
    want = 0.25 * min(np.float64(np.float32(u)) / 5.0, np.float64(np.float32(w)) * np.sqrt(2.0 / 3.0) / 1.0)
    got = m.cell_timestep(pos, vel, acc, 1.0, 2, 0.25)
    lone = m.cell_timestep(pos[:1], vel[:1], acc[:1], 1.0, 2, 0.25)
    return abs(got - want) <= 1e-15 * want and np.isinf(lone)


def pin_timestep_is_the_minimum_over_cells(m):
    """The step is the smallest cell ratio; weakening the accelerations of that cell hands the minimum to
    the next cell."""
    rng = np.random.default_rng(8)
    pos = rng.random((400, 3)).astype(np.float32)
    vel = rng.standard_normal((400, 3)).astype(np.float32)
    acc = rng.standard_normal((400, 3)).astype(np.float32)
    base = m.cell_timestep(pos, vel, acc, 1.0, 3, 0.25)
    cells = oracle.bin_cells(pos, 1.0, 3)
    ratios = []
    for c in range(27):
        i = cells == c
        if i.sum() >= 2:
            d = vel[i].astype(np.float64) - vel[i].astype(np.float64).mean(0)
            amax = np.linalg.norm(acc[i].astype(np.float64), axis=1).max()
            ratios.append((np.sqrt((d ** 2).sum() / i.sum()) / amax, c))
    ratios.sort()
    (r0, c0), (r1, _) = ratios[0], ratios[1]
    acc2 = acc.copy()
    acc2[cells == c0] /= 16   # that cell's ratio grows 16-fold: the step becomes the next smallest
    want2 = 0.25 * min(16 * r0, r1)
    got2 = m.cell_timestep(pos, vel, acc2, 1.0, 3, 0.25)
    return abs(base - 0.25 * r0) <= 1e-14 * base and abs(got2 - want2) <= 1e-14 * want2 and got2 > base


def pin_cell_max_accel_closed_form(m):
    """K=2: cell 0 holds accelerations of norm 5 (3-4-0) and 13 (5-12-0), cell 7 one of norm 1 and one of
    norm 3 (2-2-1), cell 3 one of norm 7 (2-3-6); the other five cells are empty."""
    pos = np.array([[0.1, 0.1, 0.1], [0.3, 0.2, 0.4], [0.7, 0.8, 0.9], [0.6, 0.6, 0.6], [0.2, 0.7, 0.8]],
                   np.float32)
    acc = np.array([[3, 4, 0], [5, 12, 0], [0, 0, -1], [2, -2, 1], [2, 3, 6]], np.float32)
    got = m.cell_max_accel(pos, acc, 1.0, 2)
    want = np.zeros(8)
    want[0], want[7], want[3] = 13.0, 3.0, 7.0
    return np.array_equal(got, want)


PINS = [pin_kick_closed_form, pin_drift_wraps, pin_drift_round_up_to_box_is_zero, pin_free_streaming,
        pin_second_order, pin_time_reversible, pin_momentum_conserved, pin_timestep_closed_form,
        pin_timestep_is_the_minimum_over_cells, pin_cell_max_accel_closed_form]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_kdk_pin(pin):
    assert pin(kdk_mod)


# ---------------------------------------------------------------- planted mistakes

KDK_MUTANTS = {
    "kick_sign": ("return (v + a * float(dt)).astype(np.float32)", "return (v - a * float(dt)).astype(np.float32)"),
    "full_first_kick": ("vh = kick(vel, a0.astype(np.float32), 0.5 * dt)", "vh = kick(vel, a0.astype(np.float32), dt)"),
    "drift_with_old_velocity": ("x1 = drift(pos, vh, dt, box)", "x1 = drift(pos, vel, dt, box)"),
    "second_kick_old_force": ("v1 = kick(vh, a1.astype(np.float32), 0.5 * dt)",
                              "v1 = kick(vh, a0.astype(np.float32), 0.5 * dt)"),
    "wrap_by_rounding": ("y = y - L * np.floor(y / L)", "y = y - L * np.round(y / L)"),
    "no_round_up_fix": ("f[f.astype(np.float64) >= L] = np.float32(0.0)", "pass"),
    "dispersion_not_centred": ("d = v[idx] - v[idx].mean(axis=0)", "d = v[idx]"),
    "dispersion_n_minus_1": ("sigma = np.sqrt((d ** 2).sum() / idx.size)",
                             "sigma = np.sqrt((d ** 2).sum() / (idx.size - 1))"),
    "mean_acceleration": ("amax = np.sqrt((a[idx] ** 2).sum(axis=1)).max()",
                          "amax = np.sqrt((a[idx] ** 2).sum(axis=1)).mean()"),
    "lone_particles_counted": ("if idx.size < 2:", "if idx.size < 1:"),
    "eta_dropped": ("return float(eta * best)", "return float(best)"),
    "cell_max_is_sum": ("np.maximum.at(out, cells, np.sqrt((a ** 2).sum(axis=1)))",
                        "np.add.at(out, cells, np.sqrt((a ** 2).sum(axis=1)))"),
    "cell_max_of_squares": ("np.maximum.at(out, cells, np.sqrt((a ** 2).sum(axis=1)))",
                            "np.maximum.at(out, cells, (a ** 2).sum(axis=1))"),
    "cell_max_l1": ("np.maximum.at(out, cells, np.sqrt((a ** 2).sum(axis=1)))",
                    "np.maximum.at(out, cells, np.abs(a).sum(axis=1))"),
}


def _load_variant(name, old, new):
    src = open(KDK_SRC).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType(f"oracle._kdk_mutant_{name}")
    mod.__package__ = "oracle"
    mod.__file__ = KDK_SRC
    exec(compile(src.replace(old, new), f"<kdk mutant {name}>", "exec"), mod.__dict__)
    return mod


def test_unmodified_kdk_passes_every_pin():
    assert [p.__name__ for p in PINS if not p(kdk_mod)] == []


@pytest.mark.parametrize("name", sorted(KDK_MUTANTS))
def test_kdk_planted_mistake_is_caught(name):
    m = _load_variant(name, *KDK_MUTANTS[name])
    failed = []
    for p in PINS:
        try:
            ok = p(m)
        except Exception:
            ok = False
        if not ok:
            failed.append(p.__name__)
    assert failed, f"mutant {name} passed every pin"
