"""K-sort (arXiv 1107.3622) on MI355X: Python binding of the HIP library.

The sort itself runs in libksort.so (hand-written HIP for gfx950); this
package only marshals torch tensors (device memory, streams) into the C ABI
declared in include/ksort.h.
"""
from .ksort import (  # noqa: F401
    KSORT_F32,
    KSORT_F64,
    KsortError,
    Server,
    ksort_autotune,
    ksort_f32,
    ksort_f64,
    ksort_get_default,
    ksort_partition_level,
    ksort_partition_level_exact,
    ksort_profile_enable,
    ksort_profile_read,
    ksort_release_workspaces,
    ksort_segmented,
    ksort_set_default,
    ksort_sort_ex,
    ksort_sort_exact,
    ksort_variants,
    ksort_version,
    ksort_workspace_bytes,
    load,
    sort_,
)
