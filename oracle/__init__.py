"""CPU oracle for the integer convex-hull preconditioner (arXiv 1505.00914).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline of the benchmark may import this package.  The product library under
``paper_1505_00914_amd`` never imports it and shares no code with it.
"""
from .oracle import (  # noqa: F401
    OR_OK, OR_EINVAL, OR_ERANGE, OR_EORDER, OracleError,
    build, lib_path, reduce, mask, ctz_positions, extract, chain, reduced,
    hull_chain, hull_full, precondition_and_hull, bbox, translate, auto,
    tree_levels, array_insert, tree_insert, tree_extract, hull_melkman,
    bbox_f32, quantize_f32, auto_f32, rescan_y,
    reduce_rect, precondition_and_hull_rect, translate_rect, auto_rect,
)
