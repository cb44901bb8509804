"""Pins of the oracle's counter-based RNG (Philox4x32-10) and its uniforms."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O

# Known-answer vectors published with the Random123 library (Salmon et al.,
# SC'11) for philox4x32 with 10 rounds: (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = O.philox(ctr, key)
    assert tuple(int(x) for x in got) == out


_ROCRAND_SRC = r"""
#include <cstdio>
#include <rocrand/rocrand_kernel.h>
// rocRAND's Philox4x32-10 engine: seed -> key, subsequence -> counter words
// 2,3 and offset/4 -> counter words 0,1.
int main() {
    unsigned long long seeds[3] = {0ULL, 0x0123456789abcdefULL, 211015640ULL};
    unsigned long long subs[3] = {0ULL, 5ULL, 0x100000007ULL};
    unsigned long long offs[3] = {0ULL, 4ULL * 17ULL, 4ULL * 0x1234ULL};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                rocrand_state_philox4x32_10 st;
                rocrand_init(seeds[a], subs[b], offs[c], &st);
                uint4 r = rocrand4(&st);
                printf("%llu %llu %llu %u %u %u %u\n", seeds[a], subs[b], offs[c], r.x, r.y, r.z, r.w);
            }
    return 0;
}
"""


def test_philox_matches_rocrand_engine():
    """The oracle's Philox equals rocRAND's Philox4x32-10 (a library routine,
    compiled here as host code) for several seeds, subsequences and offsets."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "ref.cpp")
        exe = os.path.join(td, "ref")
        with open(src, "w") as f:
            f.write(_ROCRAND_SRC)
        r = subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include", src, "-o", exe],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("cannot build the rocRAND reference: " + r.stderr[-300:])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    n = 0
    for line in out:
        if not line.strip():
            continue
        seed, sub, off, *w = (int(x) for x in line.split())
        q = off // 4
        ctr = (q & 0xFFFFFFFF, q >> 32, sub & 0xFFFFFFFF, sub >> 32)
        key = (seed & 0xFFFFFFFF, seed >> 32)
        assert tuple(int(x) for x in O.philox(ctr, key)) == tuple(w)
        n += 1
    assert n == 27


def test_uniform_is_open_interval_and_exact():
    lo = O.u01(0, 0)
    hi = O.u01(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 0.5 * 2.0 ** -52
    assert hi == (2.0 ** 52 - 0.5) * 2.0 ** -52
    assert 0.0 < lo < hi < 1.0
    # 52 bits: 32 from the first word, the top 20 of the second
    assert O.u01(1, 0) == (2.0 ** 20 + 0.5) * 2.0 ** -52
    assert O.u01(0, 1 << 12) == 1.5 * 2.0 ** -52
    assert O.u01(0, (1 << 12) - 1) == lo


def test_draw_schedule_uses_packet_event_block_counter():
    seed, tag = 0x0123456789ABCDEF, 7
    got = O.draw_pair(seed, tag, (5 << 32) | 3, 11, 2)
    w = O.philox((3, 5, 11, 2), (seed & 0xFFFFFFFF, (seed >> 32) ^ tag))
    assert got[0] == O.u01(int(w[0]), int(w[1]))
    assert got[1] == O.u01(int(w[2]), int(w[3]))


def test_uniforms_are_uniform():
    from scipy import stats
    u = np.array([O.draw_pair(99, 0, p, 1, 0) for p in range(4000)]).ravel()
    assert stats.kstest(u, "uniform").pvalue > 1e-3
