"""ctypes binding of libdgidp.so (include/dgidp.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.  There is no CPU fallback: if the library is not
built, importing this module raises.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library shares)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgidp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "or python paper_2607_06045_amd/build.py")

FP64, MIXED = 0, 1
DT_IDP, DT_LOWORDER = 0, 1
LIMIT_NONE, LIMIT_POSITIVITY, LIMIT_LOCAL, LIMIT_COMBINED, LIMIT_LOCAL_LOWORDER = 0, 1, 2, 3, 4
FLUX_RANOCHA, FLUX_CHANDRASHEKAR = 0, 1
BC_PERIODIC, BC_WALL, BC_CHARACTERISTIC, BC_OUTFLOW = 0, 1, 2, 3
RHS_HIGH, RHS_LOW = 0, 1
IND_HENNEMANN, IND_MLP = 0, 1
MLP_NPARAM = 5313

ERRORS = {
    -1: "DGIDP_E_INVALID_ARG", -2: "DGIDP_E_UNSUPPORTED_N", -3: "DGIDP_E_DEVICE",
    -4: "DGIDP_E_MESH_GAP_OR_OVERLAP", -5: "DGIDP_E_MESH_NOT_BALANCED",
    -6: "DGIDP_E_STATE_INADMISSIBLE", -7: "DGIDP_E_NO_MESH", -8: "DGIDP_E_NO_STATE",
    -9: "DGIDP_E_DT",
}


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("precision", ctypes.c_int), ("dt_mode", ctypes.c_int),
                ("limiter", ctypes.c_int), ("strict_dt", ctypes.c_int),
                ("volume_flux", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("fv_inadmissible", ctypes.c_int64), ("violations", ctypes.c_int64),
                ("theta_vol_min", ctypes.c_double), ("theta_mort_min", ctypes.c_double),
                ("alpha_vol_mean", ctypes.c_double), ("alpha_mort_mean", ctypes.c_double),
                ("dt", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AdaptStats(ctypes.Structure):
    _fields_ = [("n_refined", ctypes.c_int64), ("n_balance_refined", ctypes.c_int64),
                ("n_coarsened", ctypes.c_int64), ("zs_limited", ctypes.c_int64),
                ("zs_unfixable", ctypes.c_int64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _d, _i = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
_lib = ctypes.CDLL(LIB_PATH)
_SIGS = {
    "dgidp_create": (_i, [ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "dgidp_destroy": (None, [_vp]),
    "dgidp_last_error": (ctypes.c_char_p, [_vp]),
    "dgidp_set_stream": (_i, [_vp, _vp]),
    "dgidp_synchronize": (_i, [_vp]),
    "dgidp_mesh_upload": (_i, [_vp, ctypes.c_int64, _vp, _vp, _vp, _d, _d, _d, _d, _i, _i]),
    "dgidp_mesh_info": (_i, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "dgidp_set_boundaries": (_i, [_vp, _vp, _vp]),
    "dgidp_boundary_nodes": (_i, [_vp, ctypes.POINTER(ctypes.c_int64), _vp]),
    "dgidp_set_boundary_states": (_i, [_vp, _vp, _vp]),
    "dgidp_node_coords": (_i, [_vp, _vp, _vp]),
    "dgidp_state_upload": (_i, [_vp, _vp, _i]),
    "dgidp_state_download": (_i, [_vp, _vp, _i]),
    "dgidp_state_check": (_i, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "dgidp_rhs": (_i, [_vp, _i, _vp, _i]),
    "dgidp_step_noalloc": (_i, [_vp, _d]),
    "dgidp_max_dt": (_i, [_vp, _d, ctypes.POINTER(_d)]),
    "dgidp_limit": (_i, [_vp, _d, ctypes.POINTER(Stats)]),
    "dgidp_step": (_i, [_vp, _d, ctypes.POINTER(_d), ctypes.POINTER(Stats)]),
    "dgidp_step_dt": (_i, [_vp, _d, ctypes.POINTER(Stats)]),
    "dgidp_host_tables": (_i, [_i, _vp]),
    "dgidp_time_kernels": (_i, [_vp, _i, _vp]),
    "dgidp_mesh_validate": (_i, [_i, ctypes.c_int64, _vp, _vp, _vp, _i, _i,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.c_char_p, _i]),
    "dgidp_mesh_validate_bc": (_i, [_i, ctypes.c_int64, _vp, _vp, _vp, _i, _i, _vp,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_char_p, _i]),
    "dgidp_adapt_leaves": (_i, [ctypes.c_int64, _vp, _vp, _vp, _i, _i, _vp, ctypes.c_int64,
                                _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "dgidp_refine_coarsen": (_i, [_vp, _vp, _d, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(AdaptStats)]),
    "dgidp_mesh_download": (_i, [_vp, _vp, _vp, _vp]),
    "dgidp_amr_flags": (_i, [ctypes.c_int64, _vp, _vp, _i, _i, ctypes.c_float, _i,
                             ctypes.c_float, _vp]),
    "dgidp_set_graphs": (_i, [_vp, _i]),
    "dgidp_indicator": (_i, [_vp, _i, _vp, _i]),
    "dgidp_features": (_i, [_vp, _vp, _i]),
    "dgidp_mlp_set_weights": (_i, [_vp, _vp]),
    "dgidp_mlp_get_weights": (_i, [_vp, _vp]),
    "dgidp_mlp_forward": (_i, [_vp, _vp, ctypes.c_int64, _vp, _i]),
    "dgidp_mlp_grad": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_float), _i]),
    "dgidp_mlp_train_step": (_i, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_float,
                                  ctypes.POINTER(ctypes.c_float), _i]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return sorted(_SIGS)


class DgidpError(RuntimeError):
    pass


def host_tables(N):
    """The library's operator tables for degree N: dict of w, S, I, P, Wt, Vinv."""
    n = N + 1
    out = np.zeros(n + 8 * n * n)
    rc = _lib.dgidp_host_tables(N, out.ctypes.data)
    if rc:
        raise DgidpError(ERRORS.get(rc, rc))
    o = 0
    res = {}
    for key, shape in (("w", (n,)), ("S", (n, n)), ("I", (2, n, n)), ("P", (2, n, n)),
                       ("Wt", (n, 2 * n)), ("Vinv", (n, n))):
        size = int(np.prod(shape))
        res[key] = out[o:o + size].reshape(shape)
        o += size
    return res


def validate_mesh(N, level, ix, iy, nx0, ny0):
    """Host-only mesh check: returns (n_mortars, n_two_mortar_nodes) or raises."""
    level = np.ascontiguousarray(level, dtype=np.int8)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    M, T2 = ctypes.c_int64(), ctypes.c_int64()
    msg = ctypes.create_string_buffer(256)
    rc = _lib.dgidp_mesh_validate(N, len(level), level.ctypes.data, ix.ctypes.data,
                                  iy.ctypes.data, nx0, ny0, ctypes.byref(M), ctypes.byref(T2),
                                  msg, 256)
    if rc:
        raise DgidpError(f"dgidp_mesh_validate: {ERRORS.get(rc, rc)}: {msg.value.decode()}")
    return M.value, T2.value


def validate_mesh_bc(N, level, ix, iy, nx0, ny0, bc=None):
    """Host-only mesh check with side conditions bc[4] (None: all periodic):
    returns (n_mortars, n_boundary_nodes) or raises."""
    level = np.ascontiguousarray(level, dtype=np.int8)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    b = None if bc is None else np.ascontiguousarray(bc, dtype=np.int32)
    if b is not None and b.shape != (4,):
        raise DgidpError("bc must hold four conditions (x-, x+, y-, y+)")
    M, NB = ctypes.c_int64(), ctypes.c_int64()
    msg = ctypes.create_string_buffer(256)
    rc = _lib.dgidp_mesh_validate_bc(N, len(level), level.ctypes.data, ix.ctypes.data,
                                     iy.ctypes.data, nx0, ny0, None if b is None else b.ctypes.data,
                                     ctypes.byref(M), ctypes.byref(NB), msg, 256)
    if rc:
        raise DgidpError(f"dgidp_mesh_validate_bc: {ERRORS.get(rc, rc)}: {msg.value.decode()}")
    return M.value, NB.value


def adapt_leaves(level, ix, iy, nx0, ny0, flags):
    """Host-only: new leaf list after refine/coarsen flags (rules in
    include/dgidp.h).  Returns (level, ix, iy, kind, src[n, 4])."""
    level = np.ascontiguousarray(level, dtype=np.int8)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    flags = np.ascontiguousarray(flags, dtype=np.int8)
    E = len(level)
    cap = 4 * max(E, 1)
    nl, nx, ny = np.zeros(cap, np.int8), np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    kind, src = np.zeros(cap, np.int8), np.zeros((cap, 4), np.int64)
    n = ctypes.c_int64()
    rc = _lib.dgidp_adapt_leaves(E, level.ctypes.data, ix.ctypes.data, iy.ctypes.data, nx0, ny0,
                                 flags.ctypes.data, cap, nl.ctypes.data, nx.ctypes.data,
                                 ny.ctypes.data, kind.ctypes.data, src.ctypes.data, ctypes.byref(n))
    if rc:
        raise DgidpError(f"dgidp_adapt_leaves: {ERRORS.get(rc, rc)}")
    k = n.value
    return nl[:k].copy(), nx[:k].copy(), ny[:k].copy(), kind[:k].copy(), src[:k].copy()


def amr_flags(indicator, level, base_level, med_level, med_threshold, max_level, max_threshold):
    """Host-only three-level controller: refine (+1) / coarsen (-1) / keep (0)."""
    ind = np.ascontiguousarray(indicator, dtype=np.float32)
    level = np.ascontiguousarray(level, dtype=np.int8)
    flags = np.zeros(len(level), np.int8)
    rc = _lib.dgidp_amr_flags(len(level), ind.ctypes.data, level.ctypes.data, base_level,
                              med_level, med_threshold, max_level, max_threshold,
                              flags.ctypes.data)
    if rc:
        raise DgidpError(f"dgidp_amr_flags: {ERRORS.get(rc, rc)}")
    return flags


class Solver:
    """One dgidp context: a mesh, a state on the GPU and the stepping entry points."""

    def __init__(self, N=3, gamma=1.4, beta=0.1, precision=FP64, dt_mode=DT_IDP,
                 limiter=LIMIT_POSITIVITY, strict_dt=False, stream=None, volume_flux=FLUX_RANOCHA,
                 bc=None, ext=None):
        if not torch.cuda.is_available():
            raise DgidpError("dgidp needs a ROCm GPU; none is visible")
        self.N, self.n = N, N + 1
        self.gamma = gamma
        self.params = Params(N, gamma, beta, precision, dt_mode, limiter, int(strict_dt), volume_flux)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        rc = _lib.dgidp_create(ctypes.byref(self.params), _vp(self.stream.cuda_stream),
                               ctypes.byref(h))
        if rc:
            raise DgidpError(f"dgidp_create: {ERRORS.get(rc, rc)}")
        self._h = h
        self.E = self.M = self.NB = 0
        if bc is not None:
            b = np.ascontiguousarray(bc, dtype=np.int32)
            x = None if ext is None else np.ascontiguousarray(ext, dtype=np.float64).reshape(4, 4)
            self._check(_lib.dgidp_set_boundaries(self._h, b.ctypes.data,
                                                  None if x is None else x.ctypes.data),
                        "dgidp_set_boundaries")

    def close(self):
        if getattr(self, "_h", None):
            _lib.dgidp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, what):
        if rc:
            msg = _lib.dgidp_last_error(self._h).decode()
            raise DgidpError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")

    # mesh ------------------------------------------------------------------
    def set_mesh(self, level, ix, iy, x0, y0, Lx, Ly, nx0, ny0):
        level = np.ascontiguousarray(level, dtype=np.int8)
        ix = np.ascontiguousarray(ix, dtype=np.int32)
        iy = np.ascontiguousarray(iy, dtype=np.int32)
        self._check(_lib.dgidp_mesh_upload(self._h, len(level), level.ctypes.data,
                                           ix.ctypes.data, iy.ctypes.data, x0, y0, Lx, Ly,
                                           nx0, ny0), "dgidp_mesh_upload")
        E, M = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.dgidp_mesh_info(self._h, ctypes.byref(E), ctypes.byref(M)),
                    "dgidp_mesh_info")
        self.E, self.M = E.value, M.value
        nb = ctypes.c_int64()
        self._check(_lib.dgidp_boundary_nodes(self._h, ctypes.byref(nb), None), "dgidp_boundary_nodes")
        self.NB = nb.value

    def boundary_nodes(self):
        """[NB, 3] (element, face, node along the face) of every boundary node."""
        out = np.zeros((max(self.NB, 1), 3), dtype=np.int64)
        nb = ctypes.c_int64()
        self._check(_lib.dgidp_boundary_nodes(self._h, ctypes.byref(nb), out.ctypes.data),
                    "dgidp_boundary_nodes")
        return out[: nb.value]

    def set_boundary_states(self, kind, ext):
        kind = np.ascontiguousarray(kind, dtype=np.int8)
        ext = np.ascontiguousarray(ext, dtype=np.float64)
        if kind.shape != (self.NB,) or ext.shape != (self.NB, 4):
            raise DgidpError("set_boundary_states: expected kind [NB] and ext [NB, 4]")
        self._check(_lib.dgidp_set_boundary_states(self._h, kind.ctypes.data, ext.ctypes.data),
                    "dgidp_set_boundary_states")

    def node_coords(self):
        sh = (self.E, self.n, self.n)
        x, y = np.zeros(sh), np.zeros(sh)
        self._check(_lib.dgidp_node_coords(self._h, x.ctypes.data, y.ctypes.data),
                    "dgidp_node_coords")
        return x, y

    @property
    def shape(self):
        return (self.E, 4, self.n, self.n)

    # state -----------------------------------------------------------------
    def upload(self, u):
        """u: numpy array (host) or torch float64 CUDA tensor, shape [E, 4, n, n]."""
        if isinstance(u, torch.Tensor) and u.is_cuda:
            assert u.dtype == torch.float64 and tuple(u.shape) == self.shape and u.is_contiguous()
            self._check(_lib.dgidp_state_upload(self._h, u.data_ptr(), 1), "dgidp_state_upload")
        else:
            u = np.ascontiguousarray(u, dtype=np.float64)
            assert u.shape == self.shape
            self._check(_lib.dgidp_state_upload(self._h, u.ctypes.data, 0), "dgidp_state_upload")

    def download(self, device=False):
        if device:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
            self._check(_lib.dgidp_state_download(self._h, out.data_ptr(), 1),
                        "dgidp_state_download")
            return out
        out = np.zeros(self.shape)
        self._check(_lib.dgidp_state_download(self._h, out.ctypes.data, 0), "dgidp_state_download")
        return out

    def check_state(self):
        """None if the device state is admissible (finite, rho > 0, p > 0), else
        (element, node) of an inadmissible node (external element order)."""
        b = ctypes.c_int64()
        self._check(_lib.dgidp_state_check(self._h, ctypes.byref(b)), "dgidp_state_check")
        nn = self.n * self.n
        return None if b.value < 0 else (b.value // nn, b.value % nn)

    def rhs(self, which=RHS_HIGH):
        out = np.zeros(self.shape)
        self._check(_lib.dgidp_rhs(self._h, which, out.ctypes.data, 0), "dgidp_rhs")
        return out

    # time stepping -----------------------------------------------------------
    def max_dt(self, cfl):
        dt = _d()
        self._check(_lib.dgidp_max_dt(self._h, cfl, ctypes.byref(dt)), "dgidp_max_dt")
        return dt.value

    def limit(self, dt, stats=True):
        st = Stats()
        self._check(_lib.dgidp_limit(self._h, dt, ctypes.byref(st) if stats else None),
                    "dgidp_limit")
        return st.to_dict() if stats else None

    def step(self, cfl, stats=True):
        st = Stats()
        dt = _d()
        self._check(_lib.dgidp_step(self._h, cfl, ctypes.byref(dt) if stats else None,
                                    ctypes.byref(st) if stats else None), "dgidp_step")
        return st.to_dict() if stats else None

    def step_noalloc(self, cfl):
        """One SSP-RK3 step that allocates nothing (buffers in the library's
        static per-device scratch array); enqueue only."""
        self._check(_lib.dgidp_step_noalloc(self._h, cfl), "dgidp_step_noalloc")

    def step_dt(self, dt, stats=True):
        st = Stats()
        self._check(_lib.dgidp_step_dt(self._h, dt, ctypes.byref(st) if stats else None),
                    "dgidp_step_dt")
        return st.to_dict() if stats else None

    def set_graphs(self, enable):
        """Replay enqueue-only steps from a captured HIP graph (default) or not."""
        self._check(_lib.dgidp_set_graphs(self._h, int(bool(enable))), "dgidp_set_graphs")

    def time_kernels(self, reps=50):
        """Mean ms per launch of (stage kernel, mortar kernel, dt kernel), HIP events."""
        ms = np.zeros(3)
        self._check(_lib.dgidp_time_kernels(self._h, reps, ms.ctypes.data), "dgidp_time_kernels")
        return {"stage": ms[0], "mortar": ms[1], "dt": ms[2]}

    def refine_coarsen(self, flags, zs_eps=1e-10):
        """Adapt the mesh by per-leaf flags and transfer the state (Sec. 2.4)."""
        flags = np.ascontiguousarray(flags, dtype=np.int8)
        if len(flags) != self.E:
            raise ValueError("one flag per leaf")
        n = ctypes.c_int64()
        st = AdaptStats()
        self._check(_lib.dgidp_refine_coarsen(self._h, flags.ctypes.data, zs_eps, ctypes.byref(n),
                                              ctypes.byref(st)), "dgidp_refine_coarsen")
        E, M = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.dgidp_mesh_info(self._h, ctypes.byref(E), ctypes.byref(M)), "dgidp_mesh_info")
        self.E, self.M = E.value, M.value
        nb = ctypes.c_int64()
        self._check(_lib.dgidp_boundary_nodes(self._h, ctypes.byref(nb), None), "dgidp_boundary_nodes")
        self.NB = nb.value
        return st.to_dict()

    def mesh(self):
        """Current leaf list (level, ix, iy), external order."""
        lv = np.zeros(self.E, np.int8)
        ix, iy = np.zeros(self.E, np.int32), np.zeros(self.E, np.int32)
        self._check(_lib.dgidp_mesh_download(self._h, lv.ctypes.data, ix.ctypes.data, iy.ctypes.data),
                    "dgidp_mesh_download")
        return lv, ix, iy

    # ---- indicators and the learned-indicator network ----
    def indicator(self, kind=IND_HENNEMANN, device=False):
        """Per-element indicator, FP32 [E] (numpy, or a cuda tensor if device)."""
        if device:
            out = torch.empty(self.E, dtype=torch.float32, device="cuda")
            self._check(_lib.dgidp_indicator(self._h, kind, out.data_ptr(), 1), "dgidp_indicator")
            return out
        out = np.zeros(self.E, np.float32)
        self._check(_lib.dgidp_indicator(self._h, kind, out.ctypes.data, 0), "dgidp_indicator")
        return out

    def features(self, device=False):
        """The 16 learned-indicator features per element, FP32 [E, 16]."""
        if device:
            out = torch.empty((self.E, 16), dtype=torch.float32, device="cuda")
            self._check(_lib.dgidp_features(self._h, out.data_ptr(), 1), "dgidp_features")
            return out
        out = np.zeros((self.E, 16), np.float32)
        self._check(_lib.dgidp_features(self._h, out.ctypes.data, 0), "dgidp_features")
        return out

    def mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != MLP_NPARAM:
            raise ValueError(f"{MLP_NPARAM} parameters expected")
        self._check(_lib.dgidp_mlp_set_weights(self._h, w.ctypes.data), "dgidp_mlp_set_weights")

    def mlp_get_weights(self):
        w = np.zeros(MLP_NPARAM, np.float32)
        self._check(_lib.dgidp_mlp_get_weights(self._h, w.ctypes.data), "dgidp_mlp_get_weights")
        return w

    @staticmethod
    def _mlp_args(x, t=None):
        dev = isinstance(x, torch.Tensor)
        if dev:
            x = x.contiguous().float()
            if x.dim() != 2 or x.shape[1] != 16 or not x.is_cuda:
                raise ValueError("x must be a [B, 16] cuda tensor")
            if t is not None:
                t = t.contiguous().float()
                if t.shape != (x.shape[0],) or not t.is_cuda:
                    raise ValueError("t must be a [B] cuda tensor")
            return dev, x, t, x.data_ptr(), (t.data_ptr() if t is not None else None)
        x = np.ascontiguousarray(x, dtype=np.float32)
        if x.ndim != 2 or x.shape[1] != 16:
            raise ValueError("x must be [B, 16]")
        if t is not None:
            t = np.ascontiguousarray(t, dtype=np.float32)
            if t.shape != (x.shape[0],):
                raise ValueError("t must be [B]")
        return dev, x, t, x.ctypes.data, (t.ctypes.data if t is not None else None)

    def mlp_forward(self, x):
        dev, x, _, px, _ = self._mlp_args(x)
        B = x.shape[0]
        if dev:
            y = torch.empty(B, dtype=torch.float32, device="cuda")
            py = y.data_ptr()
        else:
            y = np.zeros(B, np.float32)
            py = y.ctypes.data
        self._check(_lib.dgidp_mlp_forward(self._h, px, B, py, int(dev)), "dgidp_mlp_forward")
        return y

    def mlp_grad(self, x, t):
        dev, x, t, px, pt = self._mlp_args(x, t)
        loss = ctypes.c_float()
        if dev:
            g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
            pg = g.data_ptr()
        else:
            g = np.zeros(MLP_NPARAM, np.float32)
            pg = g.ctypes.data
        self._check(_lib.dgidp_mlp_grad(self._h, px, pt, x.shape[0], pg, ctypes.byref(loss), int(dev)),
                    "dgidp_mlp_grad")
        return g, loss.value

    def mlp_train_step(self, x, t, lr):
        dev, x, t, px, pt = self._mlp_args(x, t)
        loss = ctypes.c_float()
        self._check(_lib.dgidp_mlp_train_step(self._h, px, pt, x.shape[0], lr, ctypes.byref(loss),
                                              int(dev)), "dgidp_mlp_train_step")
        return loss.value

    def synchronize(self):
        self._check(_lib.dgidp_synchronize(self._h), "dgidp_synchronize")
