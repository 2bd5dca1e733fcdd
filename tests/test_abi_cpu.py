"""The C-ABI library: loads without a GPU, exports every entry point the header
declares; its host-side operator tables agree with the oracle's independent ones."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_06045_amd", "libdgidp.so")


def declared():
    text = open(os.path.join(ROOT, "include", "dgidp.h")).read()
    return sorted(set(re.findall(r"\b(dgidp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dgidp_\w+)", out))
    missing = [s for s in declared() if s not in exported]
    assert not missing, missing
    import paper_2607_06045_amd as P
    assert sorted(P.exported_symbols()) == declared()


@pytest.mark.parametrize("N", [3, 4])
def test_library_tables_match_oracle(oracle, N):
    import paper_2607_06045_amd as P
    t = P.host_tables(N)
    xi, w, D, S = oracle.basis(N)
    I, Pm, W = oracle.mortar_ops(N)
    assert np.abs(t["w"] - w).max() < 1e-15
    assert np.abs(t["S"] - S).max() < 1e-14
    assert np.abs(t["I"] - I).max() < 1e-14
    assert np.abs(t["P"] - Pm).max() < 1e-14
    assert np.abs(t["Wt"] - W).max() < 1e-15
    assert np.array_equal(t["Wt"] > 0, W > 0)
    from oracle import indicator as IND
    assert np.abs(t["Vinv"] - np.linalg.inv(IND.vandermonde(N))).max() < 1e-13


def test_solver_refuses_without_gpu():
    import torch
    import paper_2607_06045_amd as P
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(P.DgidpError):
        P.Solver(3)


def _two_mortar_nodes(M):
    """Nodes on two mortar faces, counted from the oracle's face table."""
    faces = M.faces()
    cnt = 0
    for e in range(M.E):
        t = faces[e, :, 0] != 0
        # corners: (a=0,b=0): faces 0,2; (N,0): 1,2; (0,N): 0,3; (N,N): 1,3
        cnt += int(t[0] and t[2]) + int(t[1] and t[2]) + int(t[0] and t[3]) + int(t[1] and t[3])
    return cnt


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_mesh_validate_matches_oracle(oracle, seed):
    import paper_2607_06045_amd as P
    from workloads.meshes import random_mesh
    spec = random_mesh(seed, 4, 3, 0.4)
    M = oracle.Mesh(3, *spec.args())
    nm, n2 = P.validate_mesh(3, spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0)
    assert nm == M.M
    assert n2 == _two_mortar_nodes(M)


def test_mesh_validate_workload_counts():
    import paper_2607_06045_amd as P
    from workloads.meshes import workload_mesh
    for k, mortars in (("vortex304", 16), ("blast22k", 552), ("shear59k", 3584)):
        spec = workload_mesh(k)
        nm, _ = P.validate_mesh(3, spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0)
        assert nm == mortars


def test_mesh_validate_errors():
    import paper_2607_06045_amd as P
    lv = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 2], dtype=np.int8)
    ix = np.array([0, 0, 1, 2, 3, 3, 4, 5, 4, 5], dtype=np.int32)
    iy = np.array([0, 1, 1, 0, 0, 1, 2, 2, 3, 3], dtype=np.int32)
    with pytest.raises(P.DgidpError, match="NOT_BALANCED"):
        P.validate_mesh(3, lv, ix, iy, 2, 2)
    with pytest.raises(P.DgidpError, match="GAP_OR_OVERLAP"):
        P.validate_mesh(3, lv[:-1], ix[:-1], iy[:-1], 2, 2)
    with pytest.raises(P.DgidpError, match="GAP_OR_OVERLAP"):
        P.validate_mesh(3, np.r_[lv, 1], np.r_[ix, 0], np.r_[iy, 0], 2, 2)
    with pytest.raises(P.DgidpError, match="UNSUPPORTED_N"):
        P.validate_mesh(7, lv, ix, iy, 2, 2)
    # empty leaf list, empty root grid
    e8, e32 = np.zeros(0, np.int8), np.zeros(0, np.int32)
    with pytest.raises(P.DgidpError, match="INVALID_ARG"):
        P.validate_mesh(3, e8, e32, e32, 2, 2)
    with pytest.raises(P.DgidpError, match="INVALID_ARG"):
        P.validate_mesh(3, lv, ix, iy, 0, 2)


def test_mesh_validate_size_limits():
    """The leaf-count limit of the header (32-bit state indices): one leaf past
    2^30 / (4 (N+1)^2) is rejected before the leaves are read; a leaf above
    level 20 is outside the supported grid."""
    import paper_2607_06045_amd as P
    for N in (3, 4):
        E = (1 << 30) // (4 * (N + 1) ** 2) + 1
        lv, z = np.zeros(E, np.int8), np.zeros(E, np.int32)
        with pytest.raises(P.DgidpError, match="INVALID_ARG"):
            P.validate_mesh(N, lv, z, z, 1, 1)
    with pytest.raises(P.DgidpError, match="GAP_OR_OVERLAP"):
        P.validate_mesh(3, np.array([21], np.int8), np.zeros(1, np.int32), np.zeros(1, np.int32), 1, 1)


def test_mesh_validate_degenerate_meshes(oracle):
    """One leaf that is its own neighbour on every face (periodic 1 x 1 root),
    a 1 x 2 root, and a refined 1 x 1 root whose mortars wrap around: valid,
    and the library agrees with the oracle on the mortar count."""
    import paper_2607_06045_amd as P
    from workloads.meshes import to_spec
    cases = [to_spec((0.0, 0.0, 1.0, 1.0, 1, 1), {(0, 0, 0)}),
             to_spec((0.0, 0.0, 2.0, 1.0, 2, 1), {(0, 0, 0), (0, 1, 0)}),
             to_spec((0.0, 0.0, 1.0, 1.0, 1, 1),
                     {(1, 0, 0), (1, 1, 0), (1, 0, 1), (2, 2, 2), (2, 3, 2), (2, 2, 3), (2, 3, 3)})]
    for spec in cases:
        M, _ = P.validate_mesh(3, spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0)
        assert M == oracle.Mesh(3, *spec.args()).M


def test_mesh_validate_with_boundaries(oracle):
    """The side conditions lift the 2:1 condition across a non-periodic side: a
    2 x 1 root grid refined twice at x = 0 and not at all at x = 1 is unbalanced
    across the periodic wrap and valid between walls; the library agrees with
    the oracle on mortars and boundary nodes.  Conditions that disagree on
    periodicity across the domain, or are unknown, are rejected."""
    import paper_2607_06045_amd as P
    from workloads.meshes import random_mesh, to_spec
    leaves = {(2, i, j) for i in (0, 1) for j in range(4)} | {(1, 1, 0), (1, 1, 1), (0, 1, 0)}
    spec = to_spec((0.0, 0.0, 2.0, 1.0, 2, 1), leaves)
    a = (3, spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0)
    with pytest.raises(P.DgidpError, match="NOT_BALANCED"):
        P.validate_mesh(*a)
    with pytest.raises(P.DgidpError, match="NOT_BALANCED"):
        P.validate_mesh_bc(*a, bc=[0, 0, 0, 0])
    for bc in ([1, 1, 0, 0], [2, 3, 0, 0], [1, 1, 1, 1]):
        nm, nb = P.validate_mesh_bc(*a, bc=bc)
        M = oracle.Mesh(3, *spec.args(), bc=bc)
        assert (nm, nb) == (M.M, M.NB)
    assert P.validate_mesh_bc(*a, bc=[1, 1, 0, 0]) == (3, 20)
    assert P.validate_mesh_bc(*a, bc=[1, 1, 1, 1])[1] == 4 * (4 + 1 + 4 + 4)
    for bc in ([1, 0, 0, 0], [0, 0, 3, 0], [5, 5, 0, 0], [-1, -1, 0, 0]):
        with pytest.raises(P.DgidpError, match="INVALID_ARG"):
            P.validate_mesh_bc(*a, bc=bc)
    with pytest.raises(P.DgidpError):
        P.validate_mesh_bc(*a, bc=[1, 1, 0])
    r = random_mesh(2, 4, 3, 0.4)
    b = (3, r.level, r.ix, r.iy, r.nx0, r.ny0)
    assert P.validate_mesh_bc(*b) == (P.validate_mesh(*b)[0], 0)


def test_null_handle_is_rejected_by_every_entry_point():
    """Every entry point of include/dgidp.h that takes a context returns
    DGIDP_E_INVALID_ARG for a NULL context (and NULL or zero for the rest)
    before any device call; dgidp_destroy(NULL) is a no-op and dgidp_create
    rejects NULL parameters.  Runs without a GPU."""
    import ctypes
    from paper_2607_06045_amd import _lib
    inval = -1
    assert _lib.ERRORS[inval] == "DGIDP_E_INVALID_ARG"
    hdr = open(os.path.join(ROOT, "include", "dgidp.h")).read()
    names = sorted(set(re.findall(r"^int (dgidp_\w+)\(dgidp_ctx\* ctx", hdr, re.M)))
    assert len(names) >= 26
    ints = (ctypes.c_int, ctypes.c_int64, ctypes.c_int8, ctypes.c_int32, ctypes.c_uint64)
    for name in names:
        fn = getattr(_lib._lib, name)
        args = [0 if t in ints else 0.0 if t in (ctypes.c_double, ctypes.c_float) else None
                for t in fn.argtypes]
        assert fn(*args) == inval, name
    _lib._lib.dgidp_destroy(None)
    out = ctypes.c_void_p(7)
    assert _lib._lib.dgidp_create(None, None, ctypes.byref(out)) == inval


def test_binding_constants_match_the_header():
    """Every enumerator of include/dgidp.h that the Python binding exposes has
    the header's value (limiter modes, boundary conditions, fluxes, precision,
    time-step rules, residual kinds, indicators)."""
    import re
    import paper_2607_06045_amd as P
    from paper_2607_06045_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "dgidp.h")).read()
    enums = {}
    for body in re.findall(r"enum\s*\{([^}]*)\}", hdr):
        for name, val in re.findall(r"(DGIDP_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            enums[name] = int(val)
    checked = 0
    for name, val in enums.items():
        short = name[len("DGIDP_"):]
        for mod in (P, _lib):
            if hasattr(mod, short):
                assert getattr(mod, short) == val, (name, getattr(mod, short), val)
                checked += 1
                break
    assert checked >= 18, checked
    for short in ("LIMIT_LOCAL_LOWORDER", "BC_WALL", "BC_CHARACTERISTIC", "BC_OUTFLOW",
                  "FLUX_CHANDRASHEKAR", "LIMIT_COMBINED"):
        assert getattr(P, short) == enums["DGIDP_" + short]
