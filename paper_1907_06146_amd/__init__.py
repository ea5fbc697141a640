"""MI355X-native batched graph search for the Satellite System Graph method.

``search`` runs the paper's Alg. 1 from the nearest navigating node for a
batch of queries in the HIP library ``libssg.so`` (C ABI in include/ssg.h).
"""

from ._lib import SSGError, lib  # noqa: F401


def search(*args, **kwargs):
    """See ``binding.search``."""
    from .binding import search as _search
    return _search(*args, **kwargs)


def quantize(*args, **kwargs):
    """See ``binding.quantize``."""
    from .binding import quantize as _quantize
    return _quantize(*args, **kwargs)


def knn_graph(*args, **kwargs):
    """See ``binding.knn_graph``."""
    from .binding import knn_graph as _knn
    return _knn(*args, **kwargs)
