"""Resource check of the device code (host only, no GPU): every kernel of the
library compiles for gfx950 without scratch memory or vector-register spills.  A
spill turns into HBM traffic on every launch (a reference-capturing lambda
once pushed the matvec's per-hand arrays into scratch, tripling the river
pair's written bytes), so it is caught here rather than in a profile."""
import shutil

import pytest

from paper_2112_03804_amd import build


@pytest.mark.parametrize("source", ["pmx_device.hip", "pmx_mlp.hip"])
def test_no_scratch_or_spills(source):
    if shutil.which("hipcc") is None and not __import__("os").path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    res = build.kernel_resources(source)
    assert res, "no kernels reported"
    # SGPR spills land in VGPR lanes (no memory traffic) and are allowed
    bad = {name: r for name, r in res.items()
           if r.get("ScratchSize [bytes/lane]", "0") != "0" or r.get("VGPRs Spill", "0") != "0"}
    assert not bad, bad


def test_matvec_occupancy_targets():
    """The matvec classes reach the waves per SIMD their launch bounds ask for."""
    res = build.kernel_resources("pmx_device.hip")
    want = {"_Z5k_mvcILi512ELi3EfEv": 4, "_Z5k_mvcILi256ELi4EfEv": 3, "_Z5k_mvcILi256ELi2EfEv": 4,
            # grouped kernel: four-wide, two-wide, and four staged with two slotted (k_mvg<KH, KE, CARRY, NC, NS>)
            "_Z5k_mvgILi4ELi16ELb0ELi4ELi4EEv": 2, "_Z5k_mvgILi4ELi16ELb0ELi2ELi2EEv": 3,
            "_Z5k_mvgILi3ELi12ELb0ELi4ELi2EEv": 3, "_Z5k_mvgILi4ELi16ELb0ELi4ELi2EEv": 3,
            "_Z5k_mvgILi2ELi8ELb0ELi4ELi2EEv": 4}
    for prefix, waves in want.items():
        hits = [r for n, r in res.items() if n.startswith(prefix)]
        assert hits, prefix
        assert int(hits[0]["Occupancy [waves/SIMD]"]) >= waves, (prefix, hits[0])
