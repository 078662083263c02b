"""MI355X-native device-resident decoder for the absolute-offset block LZ77
codec of arXiv 2606.18900 (hand-written HIP kernels behind the C ABI in
include/lz.h; torch supplies device memory and streams)."""
from ._lib import LzError, lib  # noqa: F401
from .archive import Archive, SplitArchive, encode, encode_split, fasta_index, info  # noqa: F401
from .batch import Batcher  # noqa: F401
from .serve import Server  # noqa: F401,E402
from .tune import tune, tune_encoding, tune_requests  # noqa: F401,E402
