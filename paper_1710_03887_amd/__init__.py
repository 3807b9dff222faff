"""MI355X nodal discontinuous-Galerkin solver for the 3D Euler equations.

The compute path is libdg.so (hand-written HIP kernels for gfx950) behind
the C ABI declared in include/dg.h; this package is its ctypes binding with
the same function names.  Importing it fails when the library has not been
built (`python paper_1710_03887_amd/build.py`).
"""
from ._lib import *  # noqa: F401,F403
from ._lib import (Context, DGError, EXPORTED, dg_mesh_setup, dg_destroy, dg_last_error,  # noqa: F401
                   dg_sizes, dg_nodes, dg_reference_operators, dg_geometry, dg_rhs, dg_step,
                   dg_run, dg_stage, dg_last_step, dg_stable_dt, dg_prim_to_state, dg_state_to_prim,
                   dg_set_launch, Batch, MEMBERS, dg_batch_create, dg_batch_destroy,
                   dg_batch_last_error, dg_batch_run, dg_batch_first_bad, dg_batch_set_launch,
                   dg_autotune, dg_batch_autotune, dg_run_fixed, Mlp, DG_MLP_PARAMS,
                   dg_mlp_create, dg_mlp_destroy, dg_mlp_last_error, dg_mlp_get_params,
                   dg_mlp_set_params, dg_mlp_infer, dg_mlp_grad, dg_mlp_train_step,
                   dg_set_learned_bc, dg_learned_faces, dg_sample_traces, dg_set_kernel,
                   dg_get_kernel, dg_probe_setup, dg_probe_sample, dg_run_probes, dg_spectrum,
                   dg_set_damping, dg_set_curved, dg_mlp_infer_noalloc, DG_MLP_NOALLOC_ROWS)
