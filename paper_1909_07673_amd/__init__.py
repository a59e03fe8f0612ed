"""MI355X-native network-aware container scheduler (arXiv 1909.07673).

The scheduling path (criteria, TOPSIS / AHP scoring, selection, commit,
release) runs in the HIP kernels of ``libdcsched.so`` behind the C ABI of
``include/dcsched.h``; this package only marshals arguments to it.
"""
from .binding import (Scheduler, Result, RESULT_DTYPE, DcError, topsis_tiles, topsis_tiles_noalloc, lib, strerror,
                      LIB_PATH, DC_ETOOBIG, DC_STATIC_SCRATCH_BYTES,
                      DC_OK, DC_EINVAL, DC_ENOMEM, DC_EAGAIN, DC_ENOENT, DC_EDEVICE, DC_ESTATE,
                      DC_TOPSIS, DC_AHP, DC_AHP_SAATY9, DC_AHP_RATIO, DC_AHP_DIFF,
                      DC_MODE_PLAIN, DC_MODE_BATCHED, DC_MODE_SERVING, DC_ROUTE_EACH, DC_ROUTE_END,
                      DC_CRIT_CPU, DC_CRIT_RAM, DC_CRIT_ACTIVE, DC_CRIT_PATHBW, DC_CRIT_UPLINK,
                      DC_CRIT_HOPS, DEFAULT_CRIT, DC_MAX_CONTAINERS)

__all__ = [n for n in dir() if not n.startswith("_")]
