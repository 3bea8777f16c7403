"""The oracle's stream readers under AddressSanitizer and UBSan: damaged
streams (bit flips, truncation, random table and header words) must be
rejected or decoded without any out-of-bounds access or undefined
behaviour (host build of the oracle with the robustness driver)."""
import subprocess

import pytest


@pytest.mark.parametrize("seed", [11, 12])
def test_stream_readers_are_memory_safe_on_damaged_streams(seed):
    import oracle
    exe = oracle.build_fuzz_driver()
    r = subprocess.run([exe, str(seed), "150"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "damaged streams decoded" in r.stdout
