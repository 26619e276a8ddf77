"""MI355X-native constrained-RPA polarization / screened-interaction library.

The computation lives in librp.so (hand-written HIP for gfx950) behind the C
ABI declared in include/rp.h; this package is its ctypes binding plus the
per-q orchestration in `path`.  Importing it does not touch the GPU.
"""

from ._rp import (  # noqa: F401
    EXPORTED,
    STAGES,
    RP_FP64,
    RP_SPLIT_BF16,
    RP_SPLIT_BF16_X6,
    RP_W_SAMPLING,
    RP_W_TETRA,
    RP_W_TETRA_METAL,
    Context,
    RpError,
    load,
    load_tuning,
    make_cell,
    rp_chi0_accumulate,
    rp_chi0_accumulate_noalloc,
    rp_chi0_batch,
    rp_chi0_batch_graphs,
    rp_chi0_run,
    rp_head_density,
    rp_problem,
    rp_last_error,
    rp_pair_density,
    rp_profile,
    rp_profile_read,
    rp_screen_W,
    rp_screen_head,
    rp_set_tuning,
    rp_tune_entry,
    rp_synchronize,
    rp_wannier_W,
    rp_wannier_qterm,
    rp_coulomb_cell_average,
    rp_frequency_grid,
    rp_pair_grid,
    rp_plasma_frequency,
    rp_set_drude,
    rp_unfold_coef,
    rp_unfold_eps_inv,
    rp_set_fermi_level,
    rp_weights,
)
from .build import build, library_path  # noqa: F401
