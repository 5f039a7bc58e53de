"""MI355X-native real-time Kohn-Sham step (DC-MESH local field dynamics hot path).

The compute lives in the HIP library ``libdcmesh.so`` (C ABI: include/dcmesh.h);
this package binds it for torch device tensors.
"""
from .api import (  # noqa: F401
    Domain,
    Graph,
    Workspace,
    adjoint_step,
    complex_dtype,
    current,
    density,
    occupations,
    profile_collect,
    real_dtype,
    set_tuning,
    step,
    step_eq2,
    step_noalloc,
    set_tuning_shape,
    clear_tuning_shapes,
    step_maxwell,
    tuning_options,
    workspace_bytes,
)
