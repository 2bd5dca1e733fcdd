"""Oracle for the IDP-limited LGL-DGSEM on 2:1-balanced Cartesian quadtrees.

TEST INFRASTRUCTURE ONLY.  A plain FP64 CPU implementation of the method, written
from the paper (Bolm, Rueda-Ramirez, Kuzmin, Gassner: invariant-domain-preserving
limiting with AMR for LGL-DGSEM).  Only the tests, the smoke check and the CPU
baseline of the benchmark load it; the GPU library never does.  It shares no code
with the GPU library.

Parity status of each part is listed in the module docstrings of the C sources
and in the pins under tests/.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libdgo.so")
_lib = None

RHS_HIGH, RHS_LOW = 0, 1
DT_IDP, DT_LOWORDER = 0, 1
LIM_NONE, LIM_POSITIVITY, LIM_LOCAL, LIM_COMBINED, LIM_LOCAL_LO = 0, 1, 2, 3, 4
BC_PERIODIC, BC_WALL, BC_CHARACTERISTIC, BC_OUTFLOW = 0, 1, 2, 3

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _ptr(a, t=_D):
    return a.ctypes.data_as(t)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_mesh_new.restype = ctypes.c_void_p
        L.orc_mesh_new.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_char_p, ctypes.c_int]
        L.orc_mesh_new_bc.restype = ctypes.c_void_p
        L.orc_mesh_new_bc.argtypes = L.orc_mesh_new.argtypes[:11] + [ctypes.c_void_p, ctypes.c_void_p,
                                                                     ctypes.c_char_p, ctypes.c_int]
        L.orc_mesh_num_bnodes.restype = ctypes.c_int64
        L.orc_mesh_num_bnodes.argtypes = [ctypes.c_void_p]
        L.orc_mesh_boundary_nodes.argtypes = [ctypes.c_void_p, _I64]
        L.orc_mesh_set_boundary_states.restype = ctypes.c_int
        L.orc_mesh_set_boundary_states.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _D]
        L.orc_boundary_ghost.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_double, _D]
        L.orc_mesh_free.argtypes = [ctypes.c_void_p]
        L.orc_mesh_num_mortars.restype = ctypes.c_int64
        L.orc_mesh_num_mortars.argtypes = [ctypes.c_void_p]
        L.orc_mesh_set_volume_flux.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_mesh_faces.argtypes = [ctypes.c_void_p, _I64]
        L.orc_mesh_mortars.argtypes = [ctypes.c_void_p, _I64]
        L.orc_mesh_geometry.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_rhs.argtypes = [ctypes.c_void_p, _D, ctypes.c_int, ctypes.c_double, _D]
        L.orc_max_dt.restype = ctypes.c_double
        L.orc_max_dt.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double]
        L.orc_fe_step.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, _D, _D]
        L.orc_ssprk3.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        L.orc_adapt.restype = ctypes.c_int64
        L.orc_adapt.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int] * 2 + \
            [ctypes.c_void_p] * 6
        L.orc_transfer.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   _D, _D, ctypes.c_double, ctypes.c_double, _I64]
        L.orc_ssprk3_dt.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, _D]
        L.orc_basis.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.orc_mortar_ops.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_lagrange.restype = ctypes.c_double
        L.orc_lagrange.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_legendre.restype = ctypes.c_double
        L.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_flux.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_double, _D]
        L.orc_lnmean.restype = ctypes.c_double
        L.orc_lnmean.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_overlap_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.orc_theta_pressure.restype = ctypes.c_double
        L.orc_theta_pressure.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double]
        L.orc_bar_state.argtypes = [_D, _D, ctypes.c_int, ctypes.c_double, _D]
        L.orc_spec_entropy.restype = ctypes.c_double
        L.orc_spec_entropy.argtypes = [_D, ctypes.c_double]
        L.orc_theta_entropy.restype = ctypes.c_double
        L.orc_theta_entropy.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_local_bounds.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, _D, _D, _D]
        L.orc_lowsol_bounds.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, _D, _D, _D]
        L.orc_shock_indicator.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, _D]
        L.orc_fe_step_ind.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_fe_step_detail.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def adapt(level, ix, iy, nx0, ny0, flags):
    """New leaf list after refine (+1) / coarsen (-1) flags, 2:1 balanced
    (rules in dgo_amr.c).  Returns (level, ix, iy, kind, src): kind 0 kept,
    1 child, 2 parent; src [E_new, 4] old leaf ids (child: parent, child index)."""
    L = lib()
    level = np.ascontiguousarray(level, dtype=np.int8)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    flags = np.ascontiguousarray(flags, dtype=np.int8)
    E = len(level)
    cap = 4 * max(E, 1)
    nl, nx, ny = np.zeros(cap, np.int8), np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    kind, src = np.zeros(cap, np.int8), np.zeros((cap, 4), np.int64)
    n = L.orc_adapt(ctypes.c_int64(E), _ptr(level, ctypes.c_void_p), _ptr(ix, ctypes.c_void_p),
                    _ptr(iy, ctypes.c_void_p), nx0, ny0, _ptr(flags, ctypes.c_void_p),
                    _ptr(nl, ctypes.c_void_p), _ptr(nx, ctypes.c_void_p), _ptr(ny, ctypes.c_void_p),
                    _ptr(kind, ctypes.c_void_p), _ptr(src, ctypes.c_void_p))
    return nl[:n].copy(), nx[:n].copy(), ny[:n].copy(), kind[:n].copy(), src[:n].copy()


def transfer(N, kind, src, u_old, eps=1e-10, gamma=1.4):
    """Solution transfer onto the new leaves (interpolation / L2 projection),
    then the Zhang-Shu limiter with threshold eps (eps <= 0: none).  Returns
    (u_new, n_limited_groups, n_unfixable_groups)."""
    L = lib()
    kind = np.ascontiguousarray(kind, dtype=np.int8)
    src = np.ascontiguousarray(src, dtype=np.int64)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    n = N + 1
    un = np.zeros((len(kind), 4, n, n))
    counts = np.zeros(2, np.int64)
    L.orc_transfer(N, ctypes.c_int64(len(kind)), _ptr(kind, ctypes.c_void_p), _ptr(src, ctypes.c_void_p),
                   _ptr(u_old), _ptr(un), ctypes.c_double(eps), ctypes.c_double(gamma), _ptr(counts, _I64))
    return un, int(counts[0]), int(counts[1])


def set_threads(t):
    """Set the OpenMP thread count of the oracle; returns the count in effect."""
    return lib().orc_set_threads(int(t))


def basis(N):
    """LGL nodes, weights, derivative matrix D[a,k] = phi_k'(xi_a), Sbar (Sec. 2.1)."""
    n = N + 1
    xi, w = np.zeros(n), np.zeros(n)
    D, S = np.zeros((n, n)), np.zeros((n, n))
    if lib().orc_basis(N, _ptr(xi), _ptr(w), _ptr(D), _ptr(S)):
        raise ValueError(N)
    return xi, w, D, S


def mortar_ops(N):
    """Interpolation I[h,l,k], projection P[h,k,l], sparse weights Wt[k, h*n+l] (App. A)."""
    n = N + 1
    I, P, W = np.zeros((2, n, n)), np.zeros((2, n, n)), np.zeros((n, 2 * n))
    lib().orc_mortar_ops(N, _ptr(I), _ptr(P), _ptr(W))
    return I, P, W


def overlap_weights(N, scale, shift):
    """Overlap lengths of the reference face's LGL subcells with those of a face
    scaled by `scale` and shifted by `shift` (eq. local_weights)."""
    n = N + 1
    out = np.zeros((n, n))
    lib().orc_overlap_weights(N, scale, shift, _ptr(out))
    return out


def theta_pressure(u0, dc, pt, gamma):
    """Largest theta in [0,1] with rho(u0 + theta dc) > 0 and p(u0 + theta dc) >= pt."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    dc = np.ascontiguousarray(dc, dtype=np.float64)
    return lib().orc_theta_pressure(_ptr(u0), _ptr(dc), pt, gamma)


def bar_state(uL, uR, direction, gamma):
    """Bar state of the graph edge between uL (low side along direction) and uR."""
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    ub = np.zeros(4)
    lib().orc_bar_state(_ptr(uL), _ptr(uR), direction, gamma, _ptr(ub))
    return ub


def boundary_ghost(kind, ext, ui, face, gamma=1.4):
    """Ghost state of a boundary node with interior state ui on face 0..3."""
    ext = np.ascontiguousarray(ext, dtype=np.float64)
    ui = np.ascontiguousarray(ui, dtype=np.float64)
    ug = np.zeros(4)
    lib().orc_boundary_ghost(kind, _ptr(ext), _ptr(ui), face, gamma, _ptr(ug))
    return ug


def spec_entropy(u, gamma):
    """Specific entropy p rho^-gamma (0 outside the admissible set)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_spec_entropy(_ptr(u), gamma)


def theta_entropy(u0, dc, st, gamma, thi=1.0):
    """Largest theta in [0, thi] with p rho^-gamma >= st at u0 + theta dc."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    dc = np.ascontiguousarray(dc, dtype=np.float64)
    return lib().orc_theta_entropy(_ptr(u0), _ptr(dc), st, gamma, thi)


def lagrange(N, k, s):
    return lib().orc_lagrange(N, k, s)


def legendre(m, s):
    return lib().orc_legendre(m, s)


def flux(kind, uL, uR, direction, gamma):
    """kind: 'phys', 'llf', 'ranocha', 'chandrashekar'."""
    k = {"phys": 0, "llf": 1, "ranocha": 2, "chandrashekar": 3}[kind]
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    f = np.zeros(4)
    lib().orc_flux(k, _ptr(uL), _ptr(uR), direction, gamma, _ptr(f))
    return f


def lnmean(x, y):
    return lib().orc_lnmean(x, y)


STAT_KEYS = ("fv_inadmissible", "violations", "theta_vol_min", "theta_mort_min",
             "alpha_vol_mean", "alpha_mort_mean", "dt")


def _stats(a):
    d = dict(zip(STAT_KEYS, a.tolist()))
    d["fv_inadmissible"] = int(d["fv_inadmissible"])
    d["violations"] = int(d["violations"])
    return d


class Mesh:
    """A quadtree mesh in the oracle, leaves given as (level, ix, iy).  bc gives
    the condition of the sides (x-, x+, y-, y+), each BC_PERIODIC (default),
    BC_WALL, BC_CHARACTERISTIC or BC_OUTFLOW, and ext [4, 4] each side's
    exterior state (conservative); set_boundary_states overrides both per
    boundary node."""

    def __init__(self, N, level, ix, iy, x0, y0, Lx, Ly, nx0, ny0, volume_flux="ranocha",
                 bc=None, ext=None):
        self.N, self.n = N, N + 1
        self.level = np.ascontiguousarray(level, dtype=np.int8)
        self.ix = np.ascontiguousarray(ix, dtype=np.int32)
        self.iy = np.ascontiguousarray(iy, dtype=np.int32)
        self.E = len(self.level)
        self.box = (x0, y0, Lx, Ly, nx0, ny0)
        err = ctypes.create_string_buffer(256)
        self._bc = None if bc is None else np.ascontiguousarray(bc, dtype=np.int32)
        self._ext = None if ext is None else np.ascontiguousarray(ext, dtype=np.float64).reshape(4, 4)
        self._h = lib().orc_mesh_new_bc(
            N, self.E, self.level.ctypes.data, self.ix.ctypes.data, self.iy.ctypes.data, x0, y0, Lx,
            Ly, nx0, ny0, None if self._bc is None else self._bc.ctypes.data,
            None if self._ext is None else self._ext.ctypes.data, err, 256)
        if not self._h:
            raise ValueError(err.value.decode())
        self.M = lib().orc_mesh_num_mortars(self._h)
        self.NB = lib().orc_mesh_num_bnodes(self._h)
        lib().orc_mesh_set_volume_flux(self._h, {"ranocha": 0, "chandrashekar": 1}[volume_flux])

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_mesh_free(self._h)
            self._h = None

    def faces(self):
        out = np.zeros((self.E, 4, 4), dtype=np.int64)
        lib().orc_mesh_faces(self._h, _ptr(out, _I64))
        return out

    def boundary_nodes(self):
        """[NB, 3] (element, face, node along the face) of every boundary node,
        in the order of set_boundary_states."""
        out = np.zeros((max(self.NB, 1), 3), dtype=np.int64)
        lib().orc_mesh_boundary_nodes(self._h, _ptr(out, _I64))
        return out[: self.NB]

    def set_boundary_states(self, kind, ext):
        kind = np.ascontiguousarray(kind, dtype=np.int8)
        ext = np.ascontiguousarray(ext, dtype=np.float64)
        assert kind.shape == (self.NB,) and ext.shape == (self.NB, 4)
        if lib().orc_mesh_set_boundary_states(self._h, kind.ctypes.data, _ptr(ext)):
            raise ValueError("boundary condition out of range")

    def mortars(self):
        out = np.zeros((max(self.M, 1), 4), dtype=np.int64)
        lib().orc_mesh_mortars(self._h, _ptr(out, _I64))
        return out[: self.M]

    def geometry(self):
        """Node coordinates x, y and masses m, each [E, n, n] indexed (e, b, a)."""
        sh = (self.E, self.n, self.n)
        x, y, m = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        lib().orc_mesh_geometry(self._h, _ptr(x), _ptr(y), _ptr(m))
        return x, y, m

    def state_shape(self):
        return (self.E, 4, self.n, self.n)

    def rhs(self, u, which=RHS_HIGH, gamma=1.4):
        u = np.ascontiguousarray(u, dtype=np.float64)
        du = np.zeros_like(u)
        lib().orc_rhs(self._h, _ptr(u), which, gamma, _ptr(du))
        return du

    def max_dt(self, u, cfl, mode=DT_IDP, gamma=1.4):
        u = np.ascontiguousarray(u, dtype=np.float64)
        return lib().orc_max_dt(self._h, _ptr(u), cfl, mode, gamma)

    def local_bounds(self, u, gamma=1.4):
        """(rho_min, rho_max, s_min), each [E, n, n] (e, b, a), over the bar states
        of every node's low-order neighbours and the node itself."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        sh = (self.E, self.n, self.n)
        lo, hi, sm = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        lib().orc_local_bounds(self._h, _ptr(u), gamma, _ptr(lo), _ptr(hi), _ptr(sm))
        return lo, hi, sm

    def lowsol_bounds(self, ufv, gamma=1.4):
        """(rho_min, rho_max, s_min), each [E, n, n], over the low-order states
        ufv of every node and its low-order neighbours (eq. Bounds_LowOrder; s_min
        over those with positive density and pressure)."""
        ufv = np.ascontiguousarray(ufv, dtype=np.float64)
        sh = (self.E, self.n, self.n)
        lo, hi, sm = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        lib().orc_lowsol_bounds(self._h, _ptr(ufv), gamma, _ptr(lo), _ptr(hi), _ptr(sm))
        return lo, hi, sm

    def shock_indicator(self, u, gamma=1.4):
        """Per-element Hennemann indicator on the pressure, in [0, 1] (the weight of
        the local factors in combined limiting)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(self.E)
        lib().orc_shock_indicator(self._h, _ptr(u), gamma, _ptr(out))
        return out

    def fe_step(self, u, dt, gamma=1.4, beta=0.1, limiter=LIM_POSITIVITY, indicator=None):
        """One limited forward-Euler step; for LIM_COMBINED `indicator` (per
        element) replaces the computed shock indicator when given."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        st = np.zeros(len(STAT_KEYS))
        if indicator is not None:
            ind = np.ascontiguousarray(indicator, dtype=np.float64)
            rc = lib().orc_fe_step_ind(self._h, _ptr(u), dt, gamma, beta, limiter, _ptr(ind),
                                       _ptr(out), _ptr(st))
        else:
            rc = lib().orc_fe_step(self._h, _ptr(u), dt, gamma, beta, limiter, _ptr(out), _ptr(st))
        d = _stats(st)
        d["rc"] = rc
        return out, d

    def fe_step_detail(self, u, dt, gamma=1.4, beta=0.1, limiter=LIM_POSITIVITY):
        """One limited forward-Euler step with its intermediate results: returns
        (new state, stats, u_vol, dslot, theta) with u_vol the state after the
        volume limiter, dslot [M, 3n, 4] the high-order minus low-order surface
        flux terms of each mortar node (large face, lower small face, upper
        small face, each by face position) and theta [M] the mortar factors."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        uvol = np.zeros_like(u)
        M = max(self.M, 1)
        dslot = np.zeros((M, 3 * self.n, 4))
        theta = np.zeros(M)
        st = np.zeros(len(STAT_KEYS))
        rc = lib().orc_fe_step_detail(self._h, _ptr(u), dt, gamma, beta, limiter, _ptr(out), _ptr(st),
                                      _ptr(uvol), _ptr(dslot), _ptr(theta))
        d = _stats(st)
        d["rc"] = rc
        return out, d, uvol, dslot[: self.M], theta[: self.M]

    def ssprk3(self, u, cfl, mode=DT_IDP, gamma=1.4, beta=0.1, limiter=LIM_POSITIVITY):
        """One SSP-RK3 step; returns (new state, stats)."""
        u = np.array(u, dtype=np.float64, order="C", copy=True)
        st = np.zeros(len(STAT_KEYS))
        rc = lib().orc_ssprk3(self._h, _ptr(u), cfl, mode, gamma, beta, limiter, _ptr(st))
        d = _stats(st)
        d["rc"] = rc
        return u, d

    def ssprk3_dt(self, u, dt, gamma=1.4, beta=0.1, limiter=LIM_POSITIVITY):
        """One SSP-RK3 step with a given dt; returns (new state, stats)."""
        u = np.array(u, dtype=np.float64, order="C", copy=True)
        st = np.zeros(len(STAT_KEYS))
        rc = lib().orc_ssprk3_dt(self._h, _ptr(u), dt, gamma, beta, limiter, _ptr(st))
        d = _stats(st)
        d["rc"] = rc
        return u, d
