"""MI355X-native hot path of 3D SIMP compliance minimisation (PyTopo3D, arXiv 2504.05604).

The numerical work runs in ``libtopo.so`` (hand-written HIP for gfx950 behind
the C ABI in ``include/topo.h``); this package is its thin Python binding.
"""

from ._lib import (  # noqa: F401
    Batch,
    Context,
    Network,
    NotConverged,
    TopoError,
    default_opts,
    default_train_opts,
    oc_update_noalloc,
    surface_stl,
    write_stl,
    read_stl,
    voxelize,
    load,
    EXPORTED,
    LIB_PATH,
    FILTER_DENSITY,
    FILTER_SENSITIVITY,
    VOL_DESIGN,
    VOL_ALL,
    FILTER_FWD,
    FILTER_ADJ,
    FILTER_SENS,
    FILTER_VOLW,
    PREC_FP64,
    PREC_FP32,
    PREC_BF16,
    PRECOND_JACOBI,
    PRECOND_MG,
    PRECOND_LEARNED,
    KU_AUTO,
    KU_NODE,
    KU_ELEMENT,
    LOSS_REL,
    LOSS_COS,
)
