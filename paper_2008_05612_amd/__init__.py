"""MI355X-native HP-model genotype-phenotype map (arXiv 2008.05612 hot path).

Thin Python binding over the C ABI of ``libhpmap.so`` (declared in
``include/hp.h``).  Every step of the computation runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch supplies device memory
and streams.  If the library is not built, importing works but every call
raises ``LibraryMissing`` -- there is no fallback path.
"""
from ._binding import (  # noqa: F401
    FORM_BLOCKED_I8,
    FORM_GEMM_I8,
    FORM_POPCOUNT,
    NONE,
    HPError,
    Job,
    LibraryMissing,
    Structures,
    hp_components,
    hp_enumerate,
    hp_autotune,
    hp_autotune_blocked,
    hp_blocked_select,
    hp_blocked_selected,
    hp_canonical_block_count,
    hp_canonical_count,
    hp_enumerate_batch,
    hp_enumerate_batch_static,
    hp_enumerate_gap,
    hp_enumerate_symmetric,
    hp_enumerate_symmetric_blocked,
    hp_enumerate_symmetric_wide,
    hp_gemm_select,
    hp_gemm_selected,
    hp_gemm_shapes,
    hp_graph_capture_batch,
    hp_neighbors,
    hp_phi_counts,
    hp_phi_sparse,
    hp_sample,
    hp_structures,
    hp_upload,
    hp_wide_block_count,
    hp_workspace_bytes,
    library,
    library_path,
)
