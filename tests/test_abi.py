"""The C ABI without a GPU: the library loads, exports every symbol include/pcal.h
declares, plans launches on the host, and rejects invalid parameters before any
GPU call."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

pcal = pytest.importorskip("paper_2501_05993_amd.pcal")


def _declared():
    src = open(os.path.join(ROOT, "include", "pcal.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcal_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = pcal.lib()
    names = _declared()
    assert "pcal_create" in names and "pcal_extract" in names and "pcal_results" in names
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_and_codes():
    assert pcal.strerror(pcal.OK) == "ok"
    assert "invalid" in pcal.strerror(pcal.EINVAL)
    assert pcal.strerror(12345) == "unknown status"


@pytest.mark.parametrize("args", [
    (0, 1_000_000, 0, 2), (64_000_000, 0, 0, 2), (64_000_000, 3_000_000, 0, 2),
    (64_000_000, 1_000_000, -1, 2), (64_000_000, 1_000_000, 64_000_000, 2),
    (64_000_000, 1_000_000, 10_000, 4), (64_000_000, 10_000, 0, 2),  # N = 6400 > 4096
])
def test_invalid_parameters_rejected_on_host(args):
    h = ctypes.c_void_p()
    rc = pcal.lib().pcal_create(*args, 1, ctypes.byref(h))
    assert rc == pcal.EINVAL and not h.value
    with pytest.raises(pcal.PcalError):
        pcal.plan(*args)


def test_invalid_sideband_and_null_out():
    assert pcal.lib().pcal_create(64_000_000, 1_000_000, 0, 2, 0, ctypes.byref(ctypes.c_void_p())) == pcal.EINVAL
    assert pcal.lib().pcal_create(64_000_000, 1_000_000, 0, 2, 1, None) == pcal.EINVAL
    assert pcal.lib().pcal_extract(None, None, 0, None) == pcal.EINVAL
    assert pcal.lib().pcal_results(None, None, None, None) == pcal.EINVAL


@pytest.mark.parametrize("fs,fc,fo,nbits,N,R,S", [
    (16_000_000, 1_000_000, 10_000, 2, 16, 1600, 1600),       # the paper's benchmark workload
    (32_000_000, 1_000_000, 0, 2, 32, 1, 32),
    (64_000_000, 1_000_000, 10_000, 2, 64, 6400, 6400),
    (1_024_000_000, 1_000_000, 510_000, 8, 1024, 102_400, 102_400),
    (16_000_000, 1_000_000, 250_000, 2, 16, 64, 64),
    (24_000_000, 1_000_000, 500_000, 8, 24, 48, 48),
])
def test_plan_periods(fs, fc, fo, nbits, N, R, S):
    info = pcal.plan(fs, fc, fo, nbits)
    assert info["ntones"] == N
    assert info["rotator_period"] == R          # Eq. 4
    assert info["joint_period"] == S
    spv = 64 if nbits == 2 else 16
    assert info["fold_period"] % S == 0 and info["fold_period"] % spv == 0
    assert info["method"] == pcal.METHOD_PERIOD_FOLD


def test_unsupported_forms_reported():
    # a prime offset makes the joint period too long for the period fold
    with pytest.raises(pcal.PcalError) as e:
        pcal.plan(1_024_000_000, 1_000_000, 10_007, 8, method=pcal.METHOD_PERIOD_FOLD)
    assert e.value.code == pcal.ENOTSUP


def test_per_sample_forms_share_one_plan():
    """At 510 kHz (a resonator row step with |sin d| >= 0.2 at the smallest workgroup) the recurrence forms
    (direct-form resonator, coupled form) and the table form plan the same rows; the
    8-bit per-sample forms default to 768 (table) or 512 (recurrences) workgroups per launch, the 2-bit
    ones to 1024; unknown methods are rejected."""
    for nbits in (2, 8):
        forms = (pcal.METHOD_LUT, pcal.METHOD_OSC, pcal.METHOD_CFO, pcal.METHOD_MCO, pcal.METHOD_DFR_EF)
        plans = [pcal.plan(1_024_000_000, 1_000_000, 510_000, nbits, method=m) for m in forms]
        assert [p["method"] for p in plans] == list(forms)
        keys = [k for k in plans[0] if k not in ("method", "target_blocks", "device_bytes")]
        assert all(p[k] == plans[0][k] for p in plans for k in keys)
        assert [p["target_blocks"] for p in plans] == ([768] + [512] * 4 if nbits == 8 else [1024] * 5)
    with pytest.raises(pcal.PcalError) as e:
        pcal.plan(64_000_000, 1_000_000, 10_000, 2, method=7)
    assert e.value.code == pcal.EINVAL


def test_plan_device_bytes():
    """pcal_plan reports the device bytes a handle would allocate, without allocating: the fold's
    factorised tables grow with the fold period, the table form's rotator with its precision."""
    fold = pcal.plan(64_000_000, 1_000_000, 10_000, 2, method=pcal.METHOD_PERIOD_FOLD)
    M = fold["fold_period"] // 64
    assert fold["device_bytes"] > 28 * M
    lut = {p: pcal.plan(1_024_000_000, 1_000_000, 510_000, 8, method=pcal.METHOD_LUT, precision=p)["device_bytes"]
           for p in (pcal.PREC_F64, pcal.PREC_MIXED, pcal.PREC_F32)}
    R = 102_400
    assert lut[pcal.PREC_F64] - lut[pcal.PREC_MIXED] == 8 * R
    assert lut[pcal.PREC_F64] - lut[pcal.PREC_F32] == 8 * R
    osc = pcal.plan(1_024_000_000, 1_000_000, 510_000, 8, method=pcal.METHOD_OSC)["device_bytes"]
    assert lut[pcal.PREC_F64] - osc == 16 * R


@pytest.mark.parametrize("args,code", [
    ((64_000_000, 1_000_000, 10_007, 2, 1, 4096), -6),      # per-sample form needed: PCAL_ENOTSUP
    ((1 << 24, 1 << 20, 4, 2, 1, 4096), -1),                 # tables beyond the array: PCAL_EINVAL
    ((64_000_000, 1_000_000, 10_000, 2, 1, 4097), -1),       # not a multiple of the samples per byte
    ((64_000_000, 1_000_000, 10_000, 3, 1, 4096), -1),       # bad width
    ((64_000_000, 1_000_000, 10_000, 2, 0, 4096), -1),       # bad sideband
])
def test_noalloc_refused_on_the_host(args, code):
    """Refusals come from the host planner before any HIP call (no GPU needed)."""
    import ctypes

    from paper_2501_05993_amd import pcal

    fs, fc, fo, nbits, sb, ns = args
    dummy = ctypes.c_void_p(16)  # never dereferenced: the call is refused first
    assert pcal.lib().pcal_extract_noalloc(fs, fc, fo, nbits, sb, dummy, ns, dummy, None) == code

