"""Pins of the oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: a library solve (numpy/LAPACK), brute force over
every tree shape, the closed form of the discrete scheme, an invariant of the equations, an independent integrator
of the continuous model, or values printed in the literature.
"""
import copy
import dataclasses
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests import models as TM


# --------------------------------------------------------------------------------------------------------------
# Hines solve (Sec. 2: Gaussian elimination of the tree system; Sec. 4.4: operation count independent of shape)

def _dense(parent, a, b, d):
    n = len(parent)
    M = np.zeros((n, n))
    for i in range(n):
        M[i, i] = d[i]
        if i > 0:
            M[i, parent[i]] = b[i]
            M[parent[i], i] = a[i]
    return M


def _random_system(rng, parent):
    n = len(parent)
    a = -rng.uniform(0.1, 2.0, n)
    b = -rng.uniform(0.1, 2.0, n)
    a[0] = b[0] = 0.0
    d = rng.uniform(0.5, 1.5, n)
    for i in range(1, n):  # diagonal dominance as in the cable matrix: d_i >= |b_i| + sum |a_child|
        d[i] += -b[i]
        d[parent[i]] += -a[i]
    rhs = rng.normal(size=n)
    return a, b, d, rhs


def test_hines_matches_lapack_on_random_trees():
    rng = np.random.default_rng(1)
    for trial in range(300):
        n = int(rng.integers(1, 13))
        parent = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)], np.int32)
        a, b, d, rhs = _random_system(rng, parent)
        x, flops = O.hines(parent, a, b, d, rhs)
        ref = np.linalg.solve(_dense(parent, a, b, d), rhs)
        np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert flops == 8 * (n - 1) + 1


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_hines_every_tree_shape(n):
    """brute force over all (n-1)! recursive trees with n nodes"""
    rng = np.random.default_rng(n)
    count = 0
    for tail in itertools.product(*[range(i) for i in range(1, n)]):
        parent = np.array((-1,) + tail, np.int32)
        a, b, d, rhs = _random_system(rng, parent)
        x, flops = O.hines(parent, a, b, d, rhs)
        ref = np.linalg.solve(_dense(parent, a, b, d), rhs)
        np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert flops == 8 * (n - 1) + 1
        count += 1
    assert count == int(np.prod(np.arange(1, n)))


# --------------------------------------------------------------------------------------------------------------
# closed forms of the discrete scheme (Sec. 2, Eq. 1 with backward Euler)

def test_single_passive_compartment_closed_form():
    """v_n = v_inf + (v0 - v_inf) (1 + dt/tau)^-n for a passive compartment under constant current"""
    A, g, e, amp, dt = 1000.0, 1e-4, -65.0, 0.05, 0.025
    m = TM.make([[-1]], A, 0.0, {"pas": TM.pas(None, g, e), "iclamp": TM.iclamp([0], amp)}, dt=dt)
    sim = O.OracleSim(m)
    J = 100.0 * amp / A  # mA/cm^2
    v_inf = e + J / g
    tau = 1e-3 * 1.0 / g  # ms
    for n in [1, 2, 5, 40, 400, 2000]:
        sim.run_to_step(n)
        expect = v_inf + (-65.0 - v_inf) * (1.0 + dt / tau) ** (-n)
        assert abs(sim.v()[0] - expect) < 1e-11


def test_passive_chain_discrete_steady_state():
    """sealed chain with current at node 0: u_k = C cosh(mu (N - 1/2 - k)), cosh(mu) = 1 + Gm / (2 Ga)"""
    N, diam, length, g, e, amp = 30, 1.0, 20.0, 1e-4, -65.0, 0.05
    A = np.pi * diam * length
    ri = TM.ri_uniform(diam, length)
    m = TM.make([TM.chain(N)], A, ri, {"pas": TM.pas(None, g, e), "iclamp": TM.iclamp([0], amp)}, dt=10.0)
    sim = O.OracleSim(m)
    sim.run_to_step(400)
    Gm = g * A * 1e-8  # S
    Ga = 1e-6 / ri  # S
    mu = np.arccosh(1.0 + Gm / (2.0 * Ga))
    k = np.arange(N)
    C = amp * 1e-9 / ((Gm + Ga) * np.cosh(mu * (N - 0.5)) - Ga * np.cosh(mu * (N - 1.5)))
    expect = e + 1e3 * C * np.cosh(mu * (N - 0.5 - k))
    np.testing.assert_allclose(sim.v(), expect, rtol=0, atol=1e-10 * np.abs(expect - e).max())


def test_passive_cable_converges_second_order_to_continuous():
    """sealed cable of length l with current I into its end compartment converges, at the compartment centres, to
    the continuous V(x) = I r_a lambda cosh((l - x)/lambda) / sinh(l/lambda) with error O(h^2)"""
    ell, diam, ra, g, e, amp = 600.0, 1.0, 100.0, 1e-4, -65.0, 0.05  # um, um, ohm cm, S/cm^2, mV, nA
    lam = np.sqrt((1.0 / g) * (diam * 1e-4) / (4.0 * ra))  # cm
    r_a = 4.0 * ra / (np.pi * (diam * 1e-4) ** 2)  # ohm / cm
    errs = []
    for N in (15, 30, 60):
        h = ell / N
        m = TM.make([TM.chain(N)], np.pi * diam * h, TM.ri_uniform(diam, h, ra),
                    {"pas": TM.pas(None, g, e), "iclamp": TM.iclamp([0], amp)}, dt=10.0)
        sim = O.OracleSim(m)
        sim.run_to_step(600)
        x = (np.arange(N) + 0.5) * h * 1e-4  # cm
        V = 1e3 * amp * 1e-9 * r_a * lam * np.cosh((ell * 1e-4 - x) / lam) / np.sinh(ell * 1e-4 / lam)  # mV
        errs.append(np.abs(sim.v() - e - V).max())
    assert errs[2] < 1e-3 * V.max()
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4, errs


def test_passive_tree_steady_state_dense_solve():
    """steady state of a random passive tree equals the dense solve of (G_m + G_axial) u = I"""
    rng = np.random.default_rng(7)
    n = 40
    parent = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)], np.int32)
    diam = rng.uniform(0.5, 2.0, n)
    length = rng.uniform(10, 50, n)
    A = np.pi * diam * length
    ri = np.zeros(n)
    for i in range(1, n):
        p = parent[i]
        ri[i] = 1e-2 * 100.0 * ((length[i] / 2) / (np.pi * diam[i] ** 2 / 4) + (length[p] / 2) / (np.pi * diam[p] ** 2 / 4))
    nodes = np.array([0, 5, 17, 33])
    amps = np.array([0.03, -0.01, 0.02, 0.005])
    m = TM.make([parent], A, ri, {"pas": TM.pas(None, 1e-4, -65.0), "iclamp": TM.iclamp(nodes, amps)}, dt=10.0)
    sim = O.OracleSim(m)
    sim.run_to_step(500)
    G = np.diag(1e-4 * A * 1e-8)
    for i in range(1, n):
        ga = 1e-6 / ri[i]
        p = parent[i]
        G[i, i] += ga
        G[p, p] += ga
        G[i, p] -= ga
        G[p, i] -= ga
    I = np.zeros(n)
    np.add.at(I, nodes, amps * 1e-9)
    u = np.linalg.solve(G, I)
    expect = -65.0 + 1e3 * u
    np.testing.assert_allclose(sim.v(), expect, rtol=0, atol=1e-10 * np.abs(u * 1e3).max())


# --------------------------------------------------------------------------------------------------------------
# invariants

def _passive_forest(seed=3, n_cells=4, n=25):
    rng = np.random.default_rng(seed)
    off, parent, area, ri = synth._random_trees(rng, np.full(n_cells, n))
    soma = off[:-1]
    amps = rng.uniform(0.05, 0.3, n_cells)
    parents = [parent[off[c]:off[c + 1]] for c in range(n_cells)]
    m = TM.make(parents, area, ri, {"pas": TM.pas(None, 1e-4, -65.0),
                                    "iclamp": TM.iclamp(soma, amps, dl=0.3, dur=1.0)})
    return m, amps


def test_charge_balance_passive():
    """axial currents cancel in the area-weighted sum: sum_i A_i [c_i dv_i/dt + g (v_i' - e)] = 100 sum I"""
    m, amps = _passive_forest()
    sim = O.OracleSim(m)
    dt = m.dt
    on0, off0 = int(np.ceil(0.3 / dt - 0.5)), int(np.ceil(1.3 / dt - 0.5))
    v_prev = sim.v()
    for n in range(0, 80):
        sim.run_to_step(n + 1)
        v = sim.v()
        terms = m.area * (1e-3 * m.cm * (v - v_prev) / dt + 1e-4 * (v + 65.0))
        inj = 100.0 * amps.sum() if on0 <= n < off0 else 0.0
        assert abs(terms.sum() - inj) <= 1e-12 * (np.abs(terms).sum() + abs(inj) + 1e-300)
        v_prev = v


def test_rest_invariance_passive_bitwise():
    m, _ = _passive_forest()
    m.mechs.pop("iclamp")
    sim = O.OracleSim(m)
    sim.run_to_step(400)
    assert np.all(sim.v() == -65.0)


def test_hh_rest_values_and_drift():
    """HH steady-state gates at -65 mV as printed in the literature (m 0.0529, h 0.5961, n 0.3177), and a resting
    single compartment stays within 0.1 mV over 100 ms"""
    m = TM.make([[-1]], 1000.0, 0.0, {"hh": TM.hh()})
    sim = O.OracleSim(m)
    st = sim.states()
    assert abs(st["hh_m"][0] - 0.0529) < 1e-4
    assert abs(st["hh_h"][0] - 0.5961) < 1e-4
    assert abs(st["hh_n"][0] - 0.3177) < 1e-4
    sim.run(100.0)
    assert abs(sim.v()[0] + 65.0) < 0.1
    assert sim.spikes()[0].size == 0


# --------------------------------------------------------------------------------------------------------------
# an independent integrator of the continuous Hodgkin-Huxley model (RK4 at a fine step)

def _hh_rk4_spike_times(J_uA, t_end, h=1e-3):
    def rates(v):
        def vt(x, y):
            return x / np.expm1(x / y) if abs(x / y) > 1e-9 else y * (1 - x / y / 2)
        am, bm = 0.1 * vt(-(v + 40), 10), 4 * np.exp(-(v + 65) / 18)
        ah, bh = 0.07 * np.exp(-(v + 65) / 20), 1 / (np.exp(-(v + 35) / 10) + 1)
        an, bn = 0.01 * vt(-(v + 55), 10), 0.125 * np.exp(-(v + 65) / 80)
        return am, bm, ah, bh, an, bn

    def f(y):
        v, mm, hh, nn = y
        am, bm, ah, bh, an, bn = rates(v)
        i = 120 * mm ** 3 * hh * (v - 50) + 36 * nn ** 4 * (v + 77) + 0.3 * (v + 54.3)  # uA/cm^2
        return np.array([J_uA - i, am * (1 - mm) - bm * mm, ah * (1 - hh) - bh * hh, an * (1 - nn) - bn * nn])

    am, bm, ah, bh, an, bn = rates(-65.0)
    y = np.array([-65.0, am / (am + bm), ah / (ah + bh), an / (an + bn)])
    times = []
    t = 0.0
    for _ in range(int(round(t_end / h))):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y2 = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if y[0] < 0.0 <= y2[0]:
            times.append(t + h * (0.0 - y[0]) / (y2[0] - y[0]))
        y = y2
        t += h
    return np.array(times)


def _oracle_spike_times(J_uA, t_end, dt):
    A = 1000.0
    amp = J_uA * 1e-3 * A / 100.0  # nA giving J mA/cm^2 = 100 amp / A
    m = TM.make([[-1]], A, 0.0, {"hh": TM.hh(), "iclamp": TM.iclamp([0], amp)}, dt=dt)
    sim = O.OracleSim(m)
    sim.run(t_end)
    return sim.spikes()[2]


def test_hh_isi_against_rk4():
    ref = _hh_rk4_spike_times(10.0, 60.0)
    assert ref.size >= 4
    isi_ref = np.diff(ref)[1:].mean()
    assert 12.0 < isi_ref < 17.0  # literature: about 14-15 ms at 10 uA/cm^2
    errs = []
    for dt in (0.025, 0.0125):
        t = _oracle_spike_times(10.0, 60.0, dt)
        assert t.size == ref.size
        errs.append(abs(np.diff(t)[1:].mean() - isi_ref))
    assert errs[0] / isi_ref < 0.03
    assert 0.3 < errs[1] / errs[0] < 0.7  # first-order convergence of the fixed step


def _rk4_fires(J, t_end=30.0, h=2.5e-3):
    """for each step current J (uA/cm^2, from rest at -65 mV): does the continuous HH model reach 0 mV?"""
    def vt(x, y):
        small = np.abs(x / y) < 1e-9
        return np.where(small, y * (1 - x / y / 2), x / np.expm1(np.where(small, 1.0, x / y)))

    def rates(v):
        return (0.1 * vt(-(v + 40), 10), 4 * np.exp(-(v + 65) / 18), 0.07 * np.exp(-(v + 65) / 20),
                1 / (np.exp(-(v + 35) / 10) + 1), 0.01 * vt(-(v + 55), 10), 0.125 * np.exp(-(v + 65) / 80))

    def f(v, mm, hh, nn):
        am, bm, ah, bh, an, bn = rates(v)
        i = 120 * mm ** 3 * hh * (v - 50) + 36 * nn ** 4 * (v + 77) + 0.3 * (v + 54.3)
        return J - i, am * (1 - mm) - bm * mm, ah * (1 - hh) - bh * hh, an * (1 - nn) - bn * nn

    am, bm, ah, bh, an, bn = rates(np.full(J.shape, -65.0))
    y = [np.full(J.shape, -65.0), am / (am + bm), ah / (ah + bh), an / (an + bn)]
    fired = np.zeros(J.shape, bool)
    for _ in range(int(round(t_end / h))):
        k1 = f(*y)
        k2 = f(*[a + 0.5 * h * b for a, b in zip(y, k1)])
        k3 = f(*[a + 0.5 * h * b for a, b in zip(y, k2)])
        k4 = f(*[a + h * b for a, b in zip(y, k3)])
        y = [a + h / 6 * (b1 + 2 * b2 + 2 * b3 + b4) for a, b1, b2, b3, b4 in zip(y, k1, k2, k3, k4)]
        fired |= y[0] >= 0.0
    return fired


def _oracle_fires(J, t_end=30.0, dt=0.025):
    return np.array([_oracle_spike_times(j, t_end, dt).size > 0 for j in J])


def _threshold(fires, lo, hi, rounds=3, n=17):
    for _ in range(rounds):
        J = np.linspace(lo, hi, n)
        f = fires(J)
        assert not f[0] and f[-1]
        k = int(np.argmax(f))
        lo, hi = J[k - 1], J[k]
    return 0.5 * (lo + hi)


def test_hh_step_current_threshold_against_rk4():
    """the smallest step current from rest that fires the oracle's HH compartment (dt 0.025 ms) is within 2 % of
    that of the continuous model integrated by RK4"""
    ref = _threshold(_rk4_fires, 0.5, 10.0)
    got = _threshold(_oracle_fires, 0.5, 10.0)
    assert 1.0 < ref < 8.0
    assert abs(got - ref) / ref < 0.02, (got, ref)


def _hh_rates_1952(v):
    """rate constants (1/ms) of the Hodgkin-Huxley 1952 squid-axon model at 6.3 degC in the modern convention
    (rest near -65 mV), written here independently of the oracle"""
    def vt(x, y):
        return x / np.expm1(x / y) if abs(x / y) > 1e-9 else y * (1 - x / y / 2)
    return (0.1 * vt(-(v + 40), 10), 4 * np.exp(-(v + 65) / 18), 0.07 * np.exp(-(v + 65) / 20),
            1 / (np.exp(-(v + 35) / 10) + 1), 0.01 * vt(-(v + 55), 10), 0.125 * np.exp(-(v + 65) / 80))


def _clamp_step(mechs, v_from, v_to, n_steps, read, A=1000.0, dt=0.025):
    """One compartment whose huge capacitance holds v: it starts at rest at v_from, a one-step current pulse moves
    it to about v_to, and it stays there (ionic currents move it by far less than 1e-9 mV over the run). Returns
    the voltage after the pulse and read(states) after each step 1..n_steps."""
    cm = 1e12
    c = 1e-3 * cm / dt  # S/cm^2
    amp = c * (v_to - v_from) * A / 100.0  # nA
    m = TM.make([[-1]], A, 0.0, dict(mechs, iclamp=TM.iclamp([0], amp, dl=0.0, dur=dt)), cm=cm, dt=dt,
                v_init=v_from)
    sim = O.OracleSim(m)
    xs = []
    for n in range(1, n_steps + 1):
        sim.run_to_step(n)
        if n == 1:
            v1 = sim.v()[0]
        xs.append(read(sim.states()))
    assert abs(sim.v()[0] - v1) < 1e-9
    return v1, np.array(xs)


def _relaxation(x, start=2):
    """for x_{n+1} - x_inf = r (x_n - x_inf): the ratio r of successive differences (checked constant) and the
    fixed point x_inf extrapolated from the last differences"""
    x = np.asarray(x[start:], np.float64)
    dx = np.diff(x)
    # leading differences only: far above rounding and above the slow drift of the held voltage
    k = min(int(np.sum(np.abs(dx) > 1e-3 * np.abs(dx).max())), 64)
    assert k >= 8
    r = dx[1:k] / dx[:k - 1]
    assert np.abs(r - r[0]).max() < 1e-9 * max(1.0, 1.0 / (1.0 - r[0]))
    r0 = float(np.median(r))
    return r0, float(x[1] + dx[1] / (1.0 - r0))


def test_hh_gates_relax_with_the_1952_time_constants_at_clamped_voltage():
    """after a step from -65 to about -30 mV with v held, each HH gate follows x_{n+1} - x_inf = r (x_n - x_inf)
    (reading R3) with r = exp(-dt/tau), tau = 1/(alpha + beta), and settles at x_inf = alpha/(alpha + beta), both
    from the Hodgkin-Huxley 1952 rates written in this test"""
    dt = 0.025
    v, xs = _clamp_step({"hh": TM.hh()}, -65.0, -30.0, 400,
                        lambda st: [st["hh_m"][0], st["hh_h"][0], st["hh_n"][0]], dt=dt)
    assert abs(v + 30.0) < 1e-3
    am, bm, ah, bh, an, bn = _hh_rates_1952(v)
    for g, (al, be) in enumerate(((am, bm), (ah, bh), (an, bn))):
        r, x_inf = _relaxation(xs[:, g], start=2 if g else 1)
        assert abs(r - np.exp(-dt * (al + be))) < 1e-9, g
        assert abs(x_inf - al / (al + be)) < 1e-8, g


@pytest.mark.parametrize("v_from, v_to, tau_ms", [(-35.0, -65.0, 77.0), (-65.0, -35.0, 93.0)])
def test_km_relaxation_time_constant_and_half_activation(v_from, v_to, tau_ms):
    """Slow K (reading R5, an Im-like current with tau near 100 ms): under a held voltage n relaxes exponentially
    with tau close to 77 ms at -65 mV and 93 ms at -35 mV; its steady state is one half at the half-activation
    voltage -35 mV, and as a potassium activation gate it is mostly closed at rest (n_inf(-65) < 0.1) and opens with
    depolarisation"""
    dt = 0.025
    v, xs = _clamp_step({"km": synth.MechTable(node=None, params={"gbar": 2e-4})}, v_from, v_to, 300,
                        lambda st: st["km_n"][0], dt=dt)
    assert abs(v - v_to) < 1e-6
    r, n_inf = _relaxation(xs)
    tau = -dt / np.log(r)
    assert abs(tau - tau_ms) < 0.01 * tau_ms, tau
    if v_to == -35.0:
        assert abs(n_inf - 0.5) < 1e-9
        assert xs[0] < n_inf  # opening: the start (rest) value lies below
    else:
        assert n_inf < 0.1 and xs[0] > n_inf


def test_cahi_activation_and_shell_calcium_steady_state():
    """High-threshold Ca (reading R5): m is closed at rest (m_inf(-65) < 1 %), half-activated at -20 mV, and
    relaxes with tau_m = 1 ms. Calcium in a 0.1 um shell relaxes with tau_r = 80 ms toward the steady state of
    d[Ca]/dt = -i_ca / (2 F depth) - ([Ca] - [Ca]_0) / tau_r; the unit conversion is derived here in SI units, and
    an inward (negative) current must raise calcium above its resting level"""
    dt, gbar, eca, cai0, tau_r, depth_m, F = 0.025, 1e-4, 120.0, 5e-5, 80.0, 0.1e-6, 96485.33212
    mech = {"cahi": synth.MechTable(node=None, params={"gbar": gbar})}
    v, xs = _clamp_step(mech, -65.0, -20.0, 8000, lambda st: [st["cahi_m"][0], st["cahi_cai"][0]], dt=dt)
    assert abs(v + 20.0) < 1e-6
    assert xs[0, 0] < 0.5
    m0 = O.OracleSim(TM.make([[-1]], 1000.0, 0.0, dict(mech))).states()["cahi_m"][0]
    assert m0 < 0.01
    r_m, m_inf = _relaxation(xs[:200, 0], start=1)
    assert abs(r_m - np.exp(-dt / 1.0)) < 1e-9
    assert abs(m_inf - 0.5) < 1e-9
    r_c, cai_inf = _relaxation(xs[4000:, 1])
    assert abs(r_c - np.exp(-dt / tau_r)) < 1e-9
    ica = gbar * m_inf ** 2 * (v - eca)  # mA/cm^2, inward (< 0)
    assert ica < 0
    # mA/cm^2 -> A/m^2 (x10); ions into the shell per m^2 per s; mol/m^3 = mM; per s -> per ms
    rate = -(ica * 10.0) / (2.0 * F) / depth_m / 1e3  # mM/ms
    expect = cai0 + tau_r * rate
    assert expect > cai0
    assert abs(cai_inf - expect) < 1e-9 * expect


def test_expsyn_point_conductance_scaling():
    """A point conductance of G uS on a compartment of area A um^2 acts as the density 100 G / A S/cm^2 (Eq. 1:
    point currents are divided by the compartment area; 1 uS/um^2 = 100 S/cm^2). One passive compartment with a
    constant synaptic conductance (tau of 1e15 ms: no decay at double precision) follows the closed form of the
    backward-Euler recurrence toward v_inf = (g_pas e_pas + G e_syn) / (g_pas + G): the steady state checks the
    current, the rate checks the conductance on the diagonal"""
    A, gp, ep, es, w, dt = 1000.0, 1e-4, -65.0, 0.0, 1.3e-3, 0.025
    syn = synth.MechTable(node=np.array([0], np.int64), params={"tau": 1e15, "e": es})
    m = TM.make([[-1]], A, 0.0, {"pas": TM.pas(None, gp, ep), "expsyn": syn}, dt=dt,
                kick_step=np.array([0], np.int64), kick_syn=np.array([0], np.int64), kick_weight=np.array([w]))
    sim = O.OracleSim(m)
    G = w * 1e-6 / (A * 1e-8)  # S/cm^2
    v_inf = (gp * ep + G * es) / (gp + G)
    tau = 1e-3 * 1.0 / (gp + G)  # ms
    for n in [1, 2, 7, 40, 400, 4000]:
        sim.run_to_step(n)
        assert sim.states()["syn_g"][0] == w
        expect = v_inf + (ep - v_inf) * (1.0 + dt / tau) ** (-n)
        assert abs(sim.v()[0] - expect) < 1e-11, (n, sim.v()[0], expect)


# --------------------------------------------------------------------------------------------------------------
# events, batching, background streams

def _two_cell_chain(delay=2.0, w=0.05):
    """cell 0: HH compartment kicked through its synapse 0; NetCon 0 -> synapse 1 on passive cell 1"""
    syn = synth.MechTable(node=np.array([0, 1], np.int64), params={"tau": 2.0, "e": 0.0})
    mechs = {"hh": TM.hh(np.array([0], np.int64)), "pas": TM.pas(np.array([1], np.int64)), "expsyn": syn}
    return TM.make([[-1], [-1]], 1000.0, 0.0, mechs, nc_src=[0], nc_syn=np.array([1], np.int64),
                   nc_weight=np.array([w]), nc_delay=np.array([delay]), kick_step=np.array([0], np.int64),
                   kick_syn=np.array([0], np.int64), kick_weight=np.array([0.5]))


def test_event_timing_exact():
    m = _two_cell_chain()
    sim = O.OracleSim(m)
    sim.run(10.0)
    gid, step, _ = sim.spikes()
    assert gid.tolist() == [0]
    k = int(step[0])
    D = int(np.floor(2.0 / m.dt + 0.5))
    f = np.exp(-m.dt / 2.0)
    sim = O.OracleSim(m)
    sim.run_to_step(k + D)
    assert sim.states()["syn_g"][1] == 0.0
    sim.run_to_step(k + D + 1)
    assert sim.states()["syn_g"][1] == 0.05 * f
    sim.run_to_step(k + D + 41)
    assert abs(sim.states()["syn_g"][1] - 0.05 * f ** 41) <= 64 * np.finfo(float).eps * 0.05


def test_kick_arrives_at_step_zero():
    m = _two_cell_chain()
    sim = O.OracleSim(m)
    sim.run_to_step(1)
    assert sim.states()["syn_g"][0] == 0.5 * np.exp(-m.dt / 2.0)


def _small_ring(n_cells=60, n_comp=30, seed=11):
    m = synth.ring_network(n_cells=n_cells, n_comp=n_comp, seed=seed)
    m.nc_weight = m.nc_weight * 10.0  # strong enough for activity to propagate in a small ring
    return m


def test_interval_batching_equals_immediate_insertion():
    m = _small_ring()
    a = O.OracleSim(m, batch_steps=0)
    M = int(np.floor(m.nc_delay / m.dt + 0.5).min())
    b = O.OracleSim(m, batch_steps=M)
    a.run(40.0)
    b.run(40.0)
    sa, sb = a.spikes(), b.spikes()
    assert sa[0].size > 20
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert np.array_equal(a.v(), b.v())


def test_batching_rejects_interval_longer_than_min_delay():
    m = _small_ring()
    M = int(np.floor(m.nc_delay / m.dt + 0.5).min())
    with pytest.raises(ValueError):
        O.OracleSim(m, batch_steps=M + 1)


def test_determinism_and_threads():
    m = synth.cortex_50k(n_cells=40)
    runs = []
    for th in (1, 1, 4):
        s = O.OracleSim(m, n_threads=th)
        s.run(5.0)
        runs.append((s.v(), s.spikes(), s.states()["syn_g"], s.n_delivered()))
    for r in runs[1:]:
        assert np.array_equal(r[0], runs[0][0])
        for x, y in zip(r[1], runs[0][1]):
            assert np.array_equal(x, y)
        assert np.array_equal(r[2], runs[0][2])
        assert r[3] == runs[0][3]


def _permute_cells(m, perm):
    """relabel cells: new cell j is old cell perm[j]; synapses and NetCons follow their cells"""
    sizes = m.cell_sizes()[perm]
    off = np.zeros(len(perm) + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    old_nodes = np.concatenate([np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in perm])
    node_new = np.empty(m.n_comp, np.int64)
    node_new[old_nodes] = np.arange(m.n_comp)
    cell_new = np.empty(m.n_cells, np.int64)
    cell_new[perm] = np.arange(m.n_cells)
    syn = m.mechs["expsyn"]
    syn_order = np.argsort(node_new[syn.node], kind="stable")
    syn_new = np.empty_like(syn_order)
    syn_new[syn_order] = np.arange(syn_order.shape[0])
    mechs = {"hh": synth.MechTable(node=None, params=m.mechs["hh"].params),
             "expsyn": synth.MechTable(node=node_new[syn.node][syn_order], params=syn.params)}
    nc_order = np.argsort(syn_new[m.nc_syn], kind="stable")
    return synth.Model(
        n_cells=m.n_cells, cell_offset=off, parent=m.parent[old_nodes], area=m.area[old_nodes],
        ri=m.ri[old_nodes], cm=m.cm[old_nodes], v_init=m.v_init, celsius=m.celsius, mechs=mechs,
        nc_src=cell_new[m.nc_src][nc_order].astype(np.int32), nc_syn=syn_new[m.nc_syn][nc_order],
        nc_weight=m.nc_weight[nc_order], nc_delay=m.nc_delay[nc_order], threshold=m.threshold[perm],
        kick_step=m.kick_step, kick_syn=syn_new[m.kick_syn], kick_weight=m.kick_weight,
        poisson_rate_hz=0.0, poisson_weight=np.zeros(0), seed=0, dt=m.dt), node_new, cell_new


def test_cell_permutation_invariance():
    m = _small_ring(n_cells=40, n_comp=20, seed=5)
    perm = np.random.default_rng(2).permutation(m.n_cells)
    mp, node_new, cell_new = _permute_cells(m, perm)
    a, b = O.OracleSim(m), O.OracleSim(mp)
    a.run(30.0)
    b.run(30.0)
    assert np.array_equal(a.v(), b.v()[node_new])
    ga, sa, ta = a.spikes()
    gb, sb, tb = b.spikes()
    assert ga.size > 10
    key_a = sorted(zip(sa.tolist(), cell_new[ga].tolist(), ta.tolist()))
    key_b = sorted(zip(sb.tolist(), gb.tolist(), tb.tolist()))
    assert key_a == key_b


def test_spike_time_lies_in_its_step():
    m = _small_ring()
    s = O.OracleSim(m)
    s.run(30.0)
    gid, step, t = s.spikes()
    assert gid.size > 0
    assert np.all(t > (step - 1) * m.dt - 1e-12) and np.all(t <= step * m.dt + 1e-12)
    order = np.lexsort((gid, step))
    assert np.array_equal(order, np.arange(gid.size))


def test_background_event_count_and_uniformity():
    n_syn, steps = 2000, 4000
    syn = synth.MechTable(node=np.zeros(n_syn, np.int64), params={"tau": 2.0, "e": 0.0})
    m = TM.make([[-1]], 1000.0, 0.0, {"pas": TM.pas(), "expsyn": syn}, poisson_rate_hz=5.0,
                poisson_weight=np.full(n_syn, 1e-9), seed=123456789)
    s = O.OracleSim(m)
    s.run_to_step(steps)
    p = np.floor(5.0 * m.dt * 1e-3 * 2 ** 32) / 2 ** 32
    mean = n_syn * steps * p
    assert abs(s.n_delivered() - mean) < 3 * np.sqrt(mean)
    draws = np.array([O.poisson_draw(99, s_, n) for s_ in range(64) for n in range(64)], np.float64)
    hist = np.bincount((draws / 2 ** 32 * 16).astype(int), minlength=16)
    chi2 = ((hist - draws.size / 16) ** 2 / (draws.size / 16)).sum()
    assert chi2 < 37.7  # 15 degrees of freedom, p = 0.001


def test_philox_avalanche():
    """flipping one counter bit changes about half of the 128 output bits"""
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        o1 = O.philox(c, k)
        word, bit = int(rng.integers(0, 4)), int(rng.integers(0, 32))
        c2 = list(c)
        c2[word] ^= 1 << bit
        o2 = O.philox(c2, k)
        flips.append(sum(bin(a ^ b).count("1") for a, b in zip(o1, o2)))
    assert 60 < np.mean(flips) < 68


def _partitioned_run(m, parts, tstop, max_passes=80, make=None):
    """Run the cells of each partition in a model of their own, as one GPU of a sharded run would. A spike of a
    cell outside the partition reaches the partition's synapses the way the exchange at interval ends delivers it:
    as an event at step k + D with the NetCon's weight, here a kick. The partitions are rerun with the spikes of the
    previous pass until the spike lists no longer change; since every delay spans at least one interval, the run
    whose remote spikes all come from earlier intervals is that fixed point."""
    syn_node = m.mechs["expsyn"].node
    syn_cell = np.searchsorted(m.cell_offset, syn_node, side="right") - 1
    D = np.floor(m.nc_delay / m.dt + 0.5).astype(np.int64)
    n_steps = int(round(tstop / m.dt))
    prev = None
    for passes in range(1, max_passes + 1):
        spikes, v = [], np.empty(m.n_comp)
        for cells in parts:
            inside = np.zeros(m.n_cells, bool)
            inside[cells] = True
            local_syn = np.full(syn_node.shape[0], -1, np.int64)
            keep = np.nonzero(inside[syn_cell])[0]
            local_syn[keep] = np.arange(keep.shape[0])
            sub = synth.subset_cells(m, cells)
            ks, kn, kw = [sub.kick_step], [sub.kick_syn], [sub.kick_weight]
            if prev is not None:
                remote = (~inside[m.nc_src]) & inside[syn_cell[m.nc_syn]]
                for g, k in prev:
                    sel = np.nonzero(remote & (m.nc_src == g))[0]
                    ks.append(k + D[sel]); kn.append(local_syn[m.nc_syn[sel]]); kw.append(m.nc_weight[sel])
            sub = dataclasses.replace(sub, kick_step=np.concatenate(ks).astype(np.int64),
                                      kick_syn=np.concatenate(kn).astype(np.int64), kick_weight=np.concatenate(kw))
            sim = O.OracleSim(sub) if make is None else make(sub)
            sim.run_to_step(n_steps)
            gid, step, t = sim.spikes()
            spikes += [(int(cells[g]), int(k), float(x)) for g, k, x in zip(gid, step, t)]
            nodes = np.concatenate([np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in cells])
            v[nodes] = sim.v()
        spikes.sort(key=lambda s: (s[1], s[0]))
        if prev is not None and [(g, k) for g, k, _ in spikes] == prev:
            return spikes, v, passes
        prev = [(g, k) for g, k, _ in spikes]
    raise AssertionError("partitioned run did not settle")


def test_k_partition_equals_unpartitioned():
    """Sharding across devices (one spike exchange per minimum-delay interval, Sec. 2): cells split into K
    partitions that see each other's spikes only through that exchange give, bitwise, the voltages and spikes of
    the single run. Each ring synapse is fed by exactly one NetCon, so a remote event delivered as a kick is the
    same addition at the same step."""
    m = _small_ring(n_cells=40, n_comp=20, seed=5)
    a = O.OracleSim(m)
    a.run(30.0)
    g, k, t = a.spikes()
    ref = sorted(zip(k.tolist(), g.tolist(), t.tolist()))
    assert len(ref) > 10
    for K in (2, 3):
        parts = [np.arange(j, m.n_cells, K) for j in range(K)]
        spikes, v, passes = _partitioned_run(m, parts, 30.0)
        assert passes >= 3  # remote spikes changed the partitions' runs
        assert sorted((s[1], s[0], s[2]) for s in spikes) == ref
        assert np.array_equal(v, a.v())


def _active_ring(n_cells=120, n_comp=40, seed=21):
    """a small ring-recipe network with weights raised tenfold, so that spikes keep travelling between cells"""
    m = synth.ring_network(n_cells=n_cells, n_comp=n_comp, seed=seed, tstop=60.0)
    m.nc_weight = m.nc_weight * 10.0
    return m


@pytest.mark.parametrize("n0", [800, 813])
def test_checkpoint_restart_equals_one_run(n0):
    """Checkpoint-restart (Sec. 3.4): a run saved at step n0 - potentials, states, conductances and its spikes - and
    continued in a fresh model reproduces the uninterrupted run bitwise, at an interval boundary and mid-interval.
    The events in flight at n0 are rebuilt from the spikes that sent them: without those spikes the continuation
    differs, so the collapse of the queue into its firing spikes is what the equality checks."""
    m = _active_ring()
    N = 2400
    one = O.OracleSim(m, batch_steps=40)
    one.run_to_step(N)
    a = O.OracleSim(m, batch_steps=40)
    a.run_to_step(n0)
    ck = a.checkpoint()
    ga, sa, _ = a.spikes()
    in_flight = [(g, s) for g, s in zip(ga, sa) if s + 1.0 / m.dt > n0]  # sent within the shortest delay
    assert len(in_flight) > 0
    b = O.OracleSim(m, batch_steps=40)
    b.restore(ck)
    b.run_to_step(N)
    assert np.array_equal(b.v(), one.v())
    g1, s1, t1 = one.spikes()
    gb, sb, tb = b.spikes()
    after = s1 > n0
    assert np.array_equal(gb, g1[after]) and np.array_equal(sb, s1[after]) and np.array_equal(tb, t1[after])
    for k, x in one.states().items():
        assert np.array_equal(b.states()[k], x), k
    c = O.OracleSim(m, batch_steps=40)
    ck_lost = dict(ck, gid=ck["gid"][:0], spike_step=ck["spike_step"][:0])
    c.restore(ck_lost)
    c.run_to_step(N)
    assert not np.array_equal(c.v(), one.v())


def test_restart_with_new_background_streams():
    """a restart under another seed: the saved state continues with the new streams; the same as reseeding the
    uninterrupted run at the checkpoint, and different from the old streams after it"""
    m = synth.cortex_50k(n_cells=40, seed=9)
    n0, N = 400, 1200
    a = O.OracleSim(m)
    a.run_to_step(n0)
    ck = a.checkpoint()
    ref = O.OracleSim(m)
    ref.run_to_step(n0)
    ref.set_seed(777)
    ref.run_to_step(N)
    m2 = copy.copy(m)
    m2.seed = 777
    b = O.OracleSim(m2)
    b.restore(ck)
    b.run_to_step(N)
    assert np.array_equal(b.v(), ref.v())
    a.run_to_step(N)
    assert not np.array_equal(a.v(), ref.v())
    ok = O.OracleSim(m)
    with pytest.raises(RuntimeError):
        ok.run_to_step(1)
        ok.restore(ck)  # a model that has run


def test_rounding_probe_moves_each_potential_by_at_most_one_ulp():
    """the rounding-sensitivity probe (orc_set_jitter, test infrastructure for the GPU parity bar): off, it leaves the
    oracle bitwise unchanged; on, one step moves each potential by -1, 0 or +1 ulp of the unperturbed result, with
    all three outcomes present, independently of the thread count"""
    m = synth.ring_network(n_cells=30, n_comp=20, seed=4)
    plain = O.OracleSim(m)
    off = O.OracleSim(m, jitter=0)
    plain.run_to_step(40)
    off.run_to_step(40)
    assert np.array_equal(plain.v(), off.v())
    base = O.OracleSim(m)
    base.run_to_step(39)
    ck = base.checkpoint()
    ref = O.OracleSim(m)
    ref.restore(ck)
    ref.run_to_step(40)
    outs = []
    for threads in (1, 4):
        j = O.OracleSim(m, n_threads=threads, jitter=12345)
        j.restore(ck)
        j.run_to_step(40)
        outs.append(j.v())
    assert np.array_equal(outs[0], outs[1])
    v, r = outs[0], ref.v()
    up, down = np.nextafter(r, np.inf), np.nextafter(r, -np.inf)
    assert np.all((v == r) | (v == up) | (v == down))
    assert np.any(v == up) and np.any(v == down) and np.any(v == r)


def _gap_pair(amp=0.05, g_gap=0.002, areas=(1000.0, 700.0), g=1e-4, e=-65.0):
    """two single passive compartments (separate cells), a current clamp on the first, one gap junction between
    them as two half-gap instances"""
    m = TM.make([[-1], [-1]], np.array(areas), 0.0, {"pas": TM.pas(None, g, e), "iclamp": TM.iclamp([0], amp)})
    m.gap_node = np.array([0, 1], np.int64)
    m.gap_partner = np.array([1, 0], np.int64)
    m.gap_g = np.array([g_gap, g_gap])
    return m


def test_gap_junction_steady_state_of_the_coupled_pair():
    """Reading R13 at its fixed point: with v constant in time the explicit partner term and the implicit own term
    agree, so the oracle settles at the steady state of the continuous coupled pair. Written in SI units in the
    test: membrane conductance g_pas A (S/cm^2 x um^2), junction conductance G (uS), injected current I (nA):
    g_pas A_a 1e-8 (v_a - e) + G 1e-6 (v_a - v_b) = I 1e-9 and the mirror equation without I."""
    amp, G, (Aa, Ab), g, e = 0.05, 0.002, (1000.0, 700.0), 1e-4, -65.0
    m = _gap_pair(amp, G, (Aa, Ab), g, e)
    sim = O.OracleSim(m)
    sim.run_to_step(200000)  # 5 s, many membrane time constants
    gma, gmb = g * Aa * 1e-8, g * Ab * 1e-8  # S (1 um^2 = 1e-8 cm^2)
    gj = G * 1e-6  # S
    mat = np.array([[gma + gj, -gj], [-gj, gmb + gj]])
    rhs = np.array([gma * e * 1e-3 + amp * 1e-9, gmb * e * 1e-3])  # A, with e in volts
    va, vb = np.linalg.solve(mat, rhs) * 1e3  # mV
    v = sim.v()
    assert abs(v[0] - va) < 1e-9 and abs(v[1] - vb) < 1e-9, (v, va, vb)
    assert v[1] > e + 1e-3  # the coupled cell is pulled up


def test_gap_junction_one_step_is_semi_implicit():
    """One step from a state with distinct potentials: each side's own potential implicit (the junction's
    conductance on the diagonal), the partner's taken from the start of the step:
    (c + g_pas + G') (v_a' - v_a) = -g_pas (v_a - e) - G' (v_a - v_b) + J, G' = 100 G / A, c = 1e-3 cm / dt."""
    amp, G, (Aa, Ab), g, e, dt = 0.05, 0.002, (1000.0, 700.0), 1e-4, -65.0, 0.025
    m = _gap_pair(amp, G, (Aa, Ab), g, e)
    pre = O.OracleSim(m)
    pre.run_to_step(37)
    ck = pre.checkpoint()
    ck["v"] = np.array([-40.0, -70.0])
    sim = O.OracleSim(m)
    sim.restore(ck)
    sim.run_to_step(38)
    va, vb = -40.0, -70.0
    c = 1e-3 / dt
    ga, gb = 100.0 * G / Aa, 100.0 * G / Ab
    Ja = 100.0 * amp / Aa
    da = (-g * (va - e) - ga * (va - vb) + Ja) / (c + g + ga)
    db = (-g * (vb - e) - gb * (vb - va)) / (c + g + gb)
    v = sim.v()
    assert abs(v[0] - (va + da)) < 1e-12 and abs(v[1] - (vb + db)) < 1e-12, (v, va + da, vb + db)


def test_gap_junction_symmetry_and_zero_conductance():
    """two identical HH cells with identical input coupled symmetrically stay bitwise identical; a junction of zero
    conductance leaves a network bitwise unchanged"""
    cells = [TM.chain(5), TM.chain(5)]
    mechs = {"hh": TM.hh(), "iclamp": TM.iclamp([0, 5], 0.3, dl=1.0)}
    m = TM.make(cells, 800.0, 20.0, mechs)
    m.gap_node = np.array([2, 7], np.int64)
    m.gap_partner = np.array([7, 2], np.int64)
    m.gap_g = np.array([0.01, 0.01])
    sim = O.OracleSim(m)
    sim.run(30.0)
    v = sim.v()
    assert np.array_equal(v[:5], v[5:])
    g, s, _ = sim.spikes()
    assert g.size >= 2 and np.array_equal(s[g == 0], s[g == 1])
    r = synth.ring_network(n_cells=20, n_comp=15, seed=9)
    a = O.OracleSim(r)
    a.run(20.0)
    r0 = synth.add_gap_junctions(synth.ring_network(n_cells=20, n_comp=15, seed=9), g=0.0)
    assert r0.n_gap > 0
    b = O.OracleSim(r0)
    b.run(20.0)
    assert np.array_equal(a.v(), b.v())
