"""Record helpers of the qubit shared tier-2 lists on the CPU: hand-built
records, valid and with damaged count words (tests/records_check.cpp).  A
count above the list capacity must raise the list-overflow error and leave
every write inside the address's records."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which(os.environ.get("HIPCC", "hipcc")) is None, reason="hipcc not found")
def test_record_helpers_bounded(tmp_path):
    exe = tmp_path / "records_check"
    hipcc = os.environ.get("HIPCC", "hipcc")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", os.path.join(HERE, "records_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout
