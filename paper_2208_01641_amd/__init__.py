"""MI355X learned-image-codec library (HIP kernels + C++ pipeline runtime).

Python side = argument marshalling over the C ABI of liblic.so
(include/lic.h); every step of the codec runs in the library.
"""
from .codec import Codec, LicError, rans_decode, rans_encode, rans_ileave_decode, rans_ileave_encode, fnv1a  # noqa: F401
from ._lib import LAYERS, LAYER_ID  # noqa: F401
from .distill import Distill  # noqa: F401,E402
