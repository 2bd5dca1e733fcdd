"""Pins of the oracle's combined limiting (Sec. 3.5, eq. combination_posLim_local):
alpha = (1 - w) alpha_pos + w alpha_local with w the element's shock indicator on
the pressure.  The blend reduces exactly to the two pure modes at w = 0 and
w = 1; the indicator follows its modal definition; a blast keeps the
positivity bounds and conservation."""
import numpy as np
import pytest

from oracle import indicator as I
from workloads import states
from workloads.meshes import random_mesh

G = 1.4


def make(oracle, spec, N=3):
    return oracle.Mesh(N, *spec.args())


@pytest.mark.parametrize("N", [3, 4])
def test_shock_indicator_modal_definition(oracle, N):
    """C indicator against the numpy modal transform on the pressure (the
    transform itself is pinned by closed forms in test_oracle_indicator.py);
    constant pressure gives 0, a pressure that is a pure highest Legendre mode
    gives 1 (energy fraction 1 in the highest shell), and the cap of the AMR
    indicator (0.5) does not apply."""
    M = make(oracle, random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0), N)
    x, y, m = M.geometry()
    for u in (states.sedov_tophat(x, y, r0=0.5), states.random_admissible(x, 3),
              states.density_wave(x, y)):
        a, b = M.shock_indicator(u), I.shock_indicator(u, N)
        assert np.abs(a - b).max() < 1e-12
    u = states.constant(x, rho=1.2, v1=0.1, v2=0.3, p=0.7)
    assert np.all(M.shock_indicator(u) == 0.0)
    # p = 1 + 0.5 P_N(xi) P_N(eta) on every element: all energy above the
    # constant mode sits in the highest shell
    xi = np.empty_like(x)
    eta = np.empty_like(y)
    for e in range(M.E):
        x0, x1 = x[e].min(), x[e].max()
        y0, y1 = y[e].min(), y[e].max()
        xi[e] = 2 * (x[e] - x0) / (x1 - x0) - 1
        eta[e] = 2 * (y[e] - y0) / (y1 - y0) - 1
    c = np.zeros(N + 1)
    c[N] = 1.0
    pN = np.polynomial.legendre.legval(xi, c) * np.polynomial.legendre.legval(eta, c)
    u = states.conservative(np.ones_like(x), 0 * x, 0 * x, 1.0 + 0.5 * pN, G)
    w = M.shock_indicator(u)
    assert w.min() > 0.5 and w.max() <= 1.0


@pytest.mark.parametrize("seed", [0, 1])
def test_combined_reduces_to_the_pure_modes(oracle, seed):
    """w = 0 everywhere gives the positivity-limited step, w = 1 the
    locally limited one, to the last bit; a mixed w lies between them in the
    mean low-order fraction."""
    M = make(oracle, random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0))
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5) if seed == 0 else states.random_admissible(x, 7)
    dt = M.max_dt(u, 0.9)
    pos, sp = M.fe_step(u, dt, limiter=oracle.LIM_POSITIVITY)
    loc, sl = M.fe_step(u, dt, limiter=oracle.LIM_LOCAL)
    c0, s0 = M.fe_step(u, dt, limiter=oracle.LIM_COMBINED, indicator=np.zeros(M.E))
    c1, s1 = M.fe_step(u, dt, limiter=oracle.LIM_COMBINED, indicator=np.ones(M.E))
    assert np.array_equal(c0, pos) and np.array_equal(c1, loc)
    # (the mean is an OpenMP reduction: equal up to the order of the sum)
    assert abs(s0["alpha_vol_mean"] - sp["alpha_vol_mean"]) < 1e-14
    assert abs(s1["alpha_vol_mean"] - sl["alpha_vol_mean"]) < 1e-14
    w = np.random.default_rng(seed).uniform(0, 1, M.E)
    ch, sh = M.fe_step(u, dt, limiter=oracle.LIM_COMBINED, indicator=w)
    assert sp["alpha_vol_mean"] <= sh["alpha_vol_mean"] <= sl["alpha_vol_mean"]
    assert sh["violations"] == 0


def test_combined_blast_positivity_and_conservation(oracle):
    """Combined limiting with the computed indicator on a top-hat blast: the
    indicator marks the shock elements only, the positivity bounds hold after
    every stage, and mass, momentum and energy are conserved."""
    M = make(oracle, random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0))
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    w = M.shock_indicator(u)
    assert 0 < (w > 0).sum() < 0.2 * M.E
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    for _ in range(4):
        u, st = M.ssprk3(u, 0.5, limiter=oracle.LIM_COMBINED)
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0
    tot = (u * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(u) * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot - tot0) < 1e-13 * scale)
