"""Pins of the oracle's Euler fluxes: consistency, symmetry and Tadmor's entropy
conservation condition for the Ranocha two-point flux (Sec. 3 intro) and the
Chandrashekar flux (Sec. 3.6)."""
import numpy as np
import pytest

from workloads import states

GAMMAS = [1.4, 3.0, 5.0 / 3.0]


def rand_states(seed, n=50, gamma=1.4):
    x = np.zeros((n, 1, 1))
    u = states.random_admissible(x, seed, gamma=gamma, rho_range=(0.05, 3.0),
                                 p_range=(1e-3, 5.0), vmax=2.0)
    return u[:, :, 0, 0]


def entropy_vars(u, g):
    rho, m1, m2, E = u
    v1, v2 = m1 / rho, m2 / rho
    p = (g - 1) * (E - 0.5 * rho * (v1 * v1 + v2 * v2))
    s = np.log(p) - g * np.log(rho)
    return np.array([(g - s) / (g - 1) - 0.5 * rho * (v1 * v1 + v2 * v2) / p,
                     rho * v1 / p, rho * v2 / p, -rho / p])


KINDS = ["ranocha", "chandrashekar"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("g", GAMMAS)
def test_ec_flux_consistent_symmetric(oracle, g, kind):
    U = rand_states(11, gamma=g)
    for i in range(len(U)):
        for d in (0, 1):
            f = oracle.flux(kind, U[i], U[i], d, g)
            assert np.allclose(f, oracle.flux("phys", U[i], U[i], d, g), rtol=1e-13, atol=1e-13)
            j = (i + 7) % len(U)
            a = oracle.flux(kind, U[i], U[j], d, g)
            b = oracle.flux(kind, U[j], U[i], d, g)
            assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("g", GAMMAS)
def test_ec_flux_tadmor_entropy_conservation(oracle, g, kind):
    """(w_R - w_L) . f* = psi_R - psi_L with entropy S = -rho s/(gamma-1),
    potential psi = rho v_n: the flux is entropy conservative."""
    U = rand_states(12, gamma=g)
    worst = 0.0
    for i in range(len(U) - 1):
        uL, uR = U[i], U[i + 1]
        for d in (0, 1):
            f = oracle.flux(kind, uL, uR, d, g)
            lhs = (entropy_vars(uR, g) - entropy_vars(uL, g)) @ f
            rhs = uR[1 + d] - uL[1 + d]
            scale = np.abs(entropy_vars(uR, g) * f).sum() + np.abs(entropy_vars(uL, g) * f).sum()
            worst = max(worst, abs(lhs - rhs) / scale)
    assert worst < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_ec_flux_kinetic_energy_and_pressure_equilibrium(oracle, kind):
    """Constant velocity and pressure: momentum flux = v * mass flux + p, energy
    flux = mass flux |v|^2/2 + v p gamma/(gamma-1) (pressure-equilibrium preservation,
    behind the exact 0.1 : 0.2 : 0.025 error ratios of Table ConvergenceTestPositivity)."""
    g = 1.4
    v1, v2, p = 0.1, 0.2, 20.0
    for rL, rR in ((1.02, 2.97), (2.0, 2.0000001), (1.5, 0.7)):
        uL = states.conservative(np.array([rL]), np.array([v1]), np.array([v2]), np.array([p]), g)[0]
        uR = states.conservative(np.array([rR]), np.array([v1]), np.array([v2]), np.array([p]), g)[0]
        f = oracle.flux(kind, uL, uR, 0, g)
        assert abs(f[1] - (v1 * f[0] + p)) < 1e-13 * abs(f[1])
        assert abs(f[2] - v2 * f[0]) < 1e-13 * abs(f[2])
        assert abs(f[3] - (0.5 * (v1 * v1 + v2 * v2) * f[0] + v1 * p * g / (g - 1))) < 1e-12 * abs(f[3])


def test_lnmean(oracle):
    for x, y in ((1.0, 2.0), (3.0, 3.0), (1.0, 1.0 + 1e-9), (1e-7, 1.0), (5.0, 5.1)):
        ref = x if x == y else (y - x) / np.log1p((y - x) / x)
        assert abs(oracle.lnmean(x, y) - ref) <= 2e-15 * ref
    # continuity across the series threshold
    for t in (0.0199, 0.02, 0.0201):
        x, y = 1.0, (1 + t) / (1 - t)
        assert abs(oracle.lnmean(x, y) - (x - y) / np.log(x / y)) < 2e-15 * y


@pytest.mark.parametrize("g", GAMMAS)
def test_llf(oracle, g):
    U = rand_states(13, gamma=g)
    for i in range(len(U) - 1):
        for d in (0, 1):
            f = oracle.flux("llf", U[i], U[i], d, g)
            assert np.allclose(f, oracle.flux("phys", U[i], U[i], d, g), rtol=1e-14, atol=1e-14)
            uL, uR = U[i], U[i + 1]
            fl = oracle.flux("llf", uL, uR, d, g)
            fp = 0.5 * (oracle.flux("phys", uL, uR, d, g) + oracle.flux("phys", uR, uL, d, g))

            def lam(u):
                rho = u[0]
                v = u[1 + d] / rho
                p = (g - 1) * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / rho)
                return abs(v) + np.sqrt(g * p / rho)
            ref = fp - 0.5 * max(lam(uL), lam(uR)) * (uR - uL)
            assert np.allclose(fl, ref, rtol=1e-13, atol=1e-13)


def test_chandrashekar_scheme_free_stream_and_conservation(oracle):
    """The scheme with the Chandrashekar volume flux keeps a constant state and
    conserves mass, momentum and energy on a mesh with mortars."""
    from workloads.meshes import random_mesh
    spec = random_mesh(3, 4, 3, 0.4)
    M = oracle.Mesh(3, *spec.args(), volume_flux="chandrashekar")
    x, y, m = M.geometry()
    u = states.constant(x, rho=1.3, v1=0.4, v2=-0.2, p=0.9)
    assert np.abs(M.rhs(u, oracle.RHS_HIGH)).max() < 1e-12
    # per-node noise small enough that mortar interpolation stays admissible
    u = states.random_admissible(x, 5, rho_range=(0.8, 1.2), p_range=(0.8, 1.2), vmax=0.3)
    du = M.rhs(u, oracle.RHS_HIGH)
    tot = (du * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(du) * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot) < 1e-14 * scale)
    # and it is a different scheme from the Ranocha one
    R = oracle.Mesh(3, *spec.args())
    assert np.abs(R.rhs(u, oracle.RHS_HIGH) - du).max() > 1e-6 * np.abs(du).max()
