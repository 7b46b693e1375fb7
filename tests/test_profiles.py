"""The committed rocprofv3 summaries describe the current fold kernel source (CPU only).

The benchmark reports HBM traffic only while the kernel source hashes to
what the counter summary records; this keeps a kernel edit from silently
turning that figure off without fresh counters.
"""
import hashlib
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _recorded(name):
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]{16})", fh.read())
    assert m, name
    return m.group(1)


def test_fold_profiles_match_kernel_source():
    """The fold kernel's source is its body (pcal_fold.h) and its kernels (pcal_kernels.hip)."""
    h = hashlib.sha256()
    for f in ("pcal_fold.h", "pcal_kernels.hip"):
        with open(os.path.join(ROOT, "paper_2501_05993_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
    assert _recorded("fold_kernel_fold2_64M_10k_pmc.md") == sha
    assert _recorded("fold_kernel_fold2_64M_10k_trace.md") == sha


def test_profile_summaries_name_their_command():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
        assert "rocprofv3 " in text and "bench.py" in text, name
        assert len(text) < 16384, name
