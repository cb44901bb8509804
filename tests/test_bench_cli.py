"""CPU checks of the benchmark script: it refuses more than one GPU before
touching a device, and the traffic constants it reports belong to the kernel
sources the committed profile summaries were measured on (the bench line
reports traffic only while the sources still hash to them)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _profile_sha(name):
    txt = open(os.path.join(ROOT, "profiles", name)).read()
    return re.findall(r"= `([0-9a-f]{64})`", txt)


def test_traffic_constants_match_the_profile_summaries():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.K4_PROFILE["sha"] in _profile_sha("k_transport_persistent_emission_3d.md")
    assert bench.K5_PROFILE["sha"] in _profile_sha("k_chord_tau_transmission_hires.md")
