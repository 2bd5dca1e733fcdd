"""MI355X-native IDP-limited LGL-DGSEM with AMR mortars (gfx950 HIP kernels behind a C-ABI).

The compute path is libdgidp.so (include/dgidp.h); this package only binds it.
"""
from ._lib import (FP64, MIXED, DT_IDP, DT_LOWORDER, LIMIT_NONE, LIMIT_POSITIVITY, LIMIT_LOCAL, LIMIT_COMBINED,
                   LIMIT_LOCAL_LOWORDER,
                   FLUX_RANOCHA, FLUX_CHANDRASHEKAR,  # noqa: F401
                   BC_PERIODIC, BC_WALL, BC_CHARACTERISTIC, BC_OUTFLOW,
                   RHS_HIGH, RHS_LOW, DgidpError, Solver, host_tables, exported_symbols,
                   validate_mesh, validate_mesh_bc, adapt_leaves, amr_flags, IND_HENNEMANN, IND_MLP, MLP_NPARAM)
