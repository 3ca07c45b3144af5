"""MI355X-native 2D fast multipole method (arXiv:1009.3457): the M2L
translation over every box's interaction list on gfx950 matrix cores, behind
the C ABI of include/fmm2d.h (libfmm2d.so), with a thin torch binding; and
the fast Gauss transform's Hermite evaluation (include/fgt2d.h)."""
from ._binding import (  # noqa: F401
    BF16X3, F16X3, F32, F32_PASCAL, F64_HANKEL, PRECISIONS, FMMError, build_tree, fgt_hermite_coeffs, fgt_hermite_eval, gather,
    l2l, l2l_backward, l2p,
    l2p_backward, level_offset, load, m2l_backward, m2l_operators, m2m, m2m_backward, num_boxes,
    p2m, p2m_backward, p2p, p2p_backward, scatter, translation_count,
)
from ._binding import m2l as m2l_raw  # noqa: F401
from .autograd import FMMPotential, M2LFunction, m2l, potential  # noqa: F401
from .fgt import gauss_transform  # noqa: F401
