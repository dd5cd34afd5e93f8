"""MI355X-native Lloyd K-means (arxiv 2405.12052 hot path).

The clustering runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/kmeans.h (libkmeans_mi355x.so, built in-tree by build.py); this
package is its Python binding.
"""
from ._binding import (KMeans, KMeansError, FitResult, load_library, validate,  # noqa: F401
                       initnet_param_count, fit_noalloc,
                       LIB_PATH, KM_OK, KM_EINVAL, KM_ENODEV, KM_EHIP, KM_ENOMEM,
                       KM_EUNSUPPORTED, KM_OPT_GRAPH, KM_OPT_UNROLL, KM_OPT_BLOCKS,
                       KM_OPT_TIMING, KM_OPT_KEYS, KM_OPT_PERSIST, KM_OPT_WIDE,
                       KM_OPT_TRACK)
from .initnet import train as train_init_net  # noqa: F401,E402
