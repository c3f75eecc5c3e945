"""Octagonal-star screening on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``liboss.so`` (built from ``csrc/`` by
``paper_1707_05647_amd.build``) behind the C ABI of ``include/oss.h``;
``paper_1707_05647_amd._lib`` is its ctypes binding and ``screen`` a thin
convenience layer that owns torch output tensors.  Importing the package
does not load the library; the first call does, and fails loudly when the
library has not been built.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    OSS_F_ALL,
    OSS_F_GRAD,
    OSS_F_SQ,
    OSS_F_SUM,
    OSS_U8,
    OSS_U16,
    OssError,
    oss_ctx_create,
    oss_ctx_destroy,
    oss_ref_build,
    oss_ref_bytes,
    oss_ref_create,
    oss_ref_release,
    oss_ref_tables,
    oss_screen,
    oss_template_features,
)
