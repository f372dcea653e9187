"""MI355X-native (gfx950) black-box compression of strongly admissible uniform
Block Low-Rank matrices by tagging (Pearce, Yesypenko, Levitt, Martinsson,
arXiv 2501.05528).

The compute path is the HIP library ``libblrtag.so`` (C ABI in
``include/blr_tag.h``); this package is its thin binding.  Build the library
with ``python -m paper_2501_05528_amd.build``.
"""
from .api import (Batch, BlrError, Server, Operator, Plan, UBLR, basic_compress, bn_compress, bn_min_columns, colmajor, colmajor_empty, compress,  # noqa: F401
                  footprint,
                  cores, nearfield, orthonormalize, postprocess, postprocess_lowp, refine_sketch,
                  sample_bases, sketch, sketch_lowp, tag_columns, tag_rank)

__all__ = ["Batch", "Server", "footprint", "BlrError", "Operator", "Plan", "UBLR", "basic_compress", "bn_compress", "bn_min_columns", "colmajor", "colmajor_empty", "compress",
           "cores", "nearfield", "orthonormalize", "postprocess", "postprocess_lowp",
           "refine_sketch", "sample_bases", "sketch", "sketch_lowp", "tag_columns", "tag_rank"]
