"""NSGA-III environmental selection on AMD Instinct MI355X (gfx950).

Python binding of ``libnsga3.so`` (the C ABI declared in ``include/nsga3.h``).
The binding only marshals arguments: every step of the selection runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.  There
is no CPU fallback: without the built library every call raises.

    import torch, paper_2503_20286_amd as nsga3
    res = nsga3.select(objs_cuda_f32, refs_cuda_f32, K)
    res.selected, res.rank, res.niche, res.dist, res.dom_in, res.dom_out, res.info()
"""
from __future__ import annotations

from ._native import (  # noqa: F401
    ASSOC_BF16, ASSOC_FP32, NICHING_EXACT, NICHING_ONESHOT, NUM_PHASES, PHASES, Context, Info,
    NativeError, Plan, Selection, STATUS, default_context, exported_symbols, header_symbols, lib_path, load, select, version,
    workspace_size, select_noalloc, alloc_outputs, rvea_select, RveaSelection,
    hype_select, HypeSelection, sbx_pm, gather_rows,
    OK, E_INVALID, E_NONFINITE, E_NOMEM, E_HIP, E_UNSUPPORTED,
)

__all__ = ["select", "Context", "Plan", "Selection", "Info", "NativeError", "load", "version",
           "ASSOC_FP32", "ASSOC_BF16", "NICHING_EXACT", "NICHING_ONESHOT", "rvea_select", "hype_select", "sbx_pm", "gather_rows"]
