"""histmi: exact 256-bin histograms of packed 8-bit pixel streams on MI355X (gfx950).

The compute path is libhistmi.so (HIP kernels + C ABI, see include/histmi.h); this package
is its thin binding.  There is no CPU fallback: calls fail if the library is not built.
"""

from ._lib import (  # noqa: F401
    AUTO_FLAT_R, EBUSY, ECANCELED, EDEVICE, EINVAL, ENOMEM, ENOTSUP, EOVERFLOW, ETIMEDOUT, OK,
    MODE_AHIST, MODE_AUTO, MODE_WAVEAGG, MODE_WAVEHIST, PAT_FLAT, PAT_IDENTITY, PAT_PAPER960, RMAX_MAX, S_MAX,
    BatchGraph, HistError, Ingest, Pattern, Server, Stream, declared_symbols, device_info, diag, hist_batch, hist_u8,
    hist_u8_noalloc, hist_u8_u64, load, pattern_init, pattern_update, pattern_validate, strerror, tune_get, tune_set,
    set_wait_limits,
    TUNE_STREAM, TUNE_STREAM_KNOWN, read_probe, CRIT_MAXBIN, CRIT_COLLISION, CRIT_BOTH,
)
from ._lib import LIB_PATH  # noqa: F401
