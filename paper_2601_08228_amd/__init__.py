"""MI355X (gfx950) w-product library: lazy lifting transforms and lifting with
chosen predict / update stencils, face-product GEMMs on MFMA, w-svd by
one-sided Jacobi, the pseudo-inverse, and the reverse-mode derivative.

Importing the package loads nothing; the HIP library is loaded on the first
call and a missing build raises ImportError.
"""

from .wprod import (  # noqa: F401
    w_transform, w_itransform, w_transform_adj, w_itransform_adj, w_transform_split,
    w_itransform_adj_split, w_face_product, w_face_product_split, w_face_product_gemm,
    w_face_product_workspace, w_product, w_product_workspace, w_product_noalloc,
    w_product_noalloc_scratch_bytes, w_svd, w_svd_timed,
    w_svd_workspace, w_svd_sparse, w_svd_sparse_workspace,
    SvdResult, w_pinv, w_pinv_workspace, w_transform_scheme, w_transform_scheme_split,
    w_product_scheme, w_product_scheme_workspace,
)
from .autograd import WProduct, w_product_ad  # noqa: F401
from . import deblur, schemes, synth  # noqa: F401
