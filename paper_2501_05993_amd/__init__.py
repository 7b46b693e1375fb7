"""MI355X (gfx950) implementation of fast multi-tone phase-calibration extraction.

The work runs in ``libpcal.so`` (HIP kernels behind the C ABI of
``include/pcal.h``); :mod:`.pcal` is its thin Python binding.
"""
from .pcal import (EAGAIN, EHIP, EINVAL, ENOMEM, ENOTSUP, ESTATE, METHOD_AUTO, METHOD_LUT,  # noqa: F401
                   METHOD_OSC, METHOD_PERIOD_FOLD, OK, PREC_F32, PREC_F64, PREC_MIXED, PCal, PCalBatch, PCalServer,
                   PcalError,
                   lib, plan, plan_launch, strerror)
