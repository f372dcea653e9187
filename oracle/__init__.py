"""Plain FP64 CPU oracle for tagged uniform-BLR compression.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP library is checked against.  Only the test suite,
the package smoke check and the benchmark's ``cpu_baseline`` leg may import
it; the product path never does, and it shares no code with the library
(neither imports the other; both consume arrays from ``workloads``).

Every function follows the paper's statement of the step it implements
(section, equation or algorithm cited in its docstring) in the paper's order
and notation, with numpy/scipy library primitives (matmul, SVD, LP solver)
as steps.  Readings of points the paper leaves open are marked "Reading:".

Modules
-------
admissibility   near/far lists and probe colours (Section 2.5, Section 6.1)
operators       black-box operators: dense matrix and kernel matrices
tagging         Alg. 2 (tagging) with the aspect-ratio optimisation of Section 5.3
reconstruct     steps (II)-(III) of Table 1, the uBLR apply, error metrics
refine          mixed-precision tagging with one FP64 refinement sketch (not in the paper)
basic           Alg. 3 (basic randomized SVD per box), the paper's benchmark for step (I)
bn              Alg. 1 (block nullification), the method tagging improves on
rank            tolerance-driven choice of the uniform rank from the tagged samples
truncate        per-box ranks from a tolerance by truncating a computed representation
"""
from . import admissibility, operators, tagging, reconstruct, refine, basic, bn, rank, truncate  # noqa: F401
from .admissibility import near_lists, far_lists, colours, greedy_colours, lists_and_colours, num_tag_columns  # noqa: F401
from .operators import DenseOperator, KernelOperator, CountingOperator  # noqa: F401
from .tagging import (extended_test_matrix, null_space, projected_tags, aspect_ratio,  # noqa: F401
                      optimise_tag_vector, tag_plan, tag_postprocess, col_topk, tag_bases)
from .reconstruct import (cores, nearfield_probes, ublr_apply, dense_reconstruction,  # noqa: F401
                          rel_fro_error, power_norm_estimate, reconstruct_tag)
from .refine import (sample_basis, sample_bases, mixed_test_blocks, far_sample,  # noqa: F401
                     refine_bases, reconstruct_tag_refined)
from .basic import masked_test_matrix, basic_bases, reconstruct_basic  # noqa: F401
from .bn import bn_columns, neighbour_rows, null_r, bn_bases, reconstruct_bn  # noqa: F401
from .rank import box_singular_values, rank_for_tolerance  # noqa: F401
from .truncate import representation_norm, truncate_ublr  # noqa: F401
