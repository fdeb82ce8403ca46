"""MI355X-native variable-coefficient Stokes solver (MAC grid, FGMRES + multigrid).

The compute path is the HIP library ``libstokes.so`` built from ``csrc/``; this
package only marshals arguments to its C-ABI (``include/stokes.h``).  There is
no CPU fallback: importing the binding without the built library raises.
"""
from ._binding import (  # noqa: F401
    STATUS_NAMES,
    StokesError,
    StokesGrid,
    StokesOptions,
    StokesStats,
    StokesSolver,
    UNet,
    stokes_attach_learned,
    stokes_learned_tuple,
    library_path,
    load_library,
    stokes_apply,
    stokes_default_options,
    stokes_destroy,
    stokes_last_error,
    stokes_profile_kernel,
    stokes_profile_read,
    stokes_setup,
    stokes_solve,
    stokes_stream_copy,
    StokesFluids,
    MAX_SOLIDS,
    make_fluids,
    stokes_coefficients,
    StokesBody,
    stokes_explicit_rhs,
    make_body,
    stokes_rigid_workspace_size,
    stokes_rigid_projection,
    stokes_workspace_size,
    stokes_unet_param_count,
    stokes_unet_forward_flops,
    stokes_unet_workspace_size,
)
