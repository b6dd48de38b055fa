"""Pins for the oracle's Philox4x32-10 / Box-Muller generator."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

# Known-answer vectors distributed with the Random123 reference implementation
# of Philox4x32-10 (Salmon et al., SC'11): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    out = philox.philox4x32_10(*ctr, *key)
    assert tuple(int(x) for x in out) == expect


ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0), stream = strtoull(argv[2], 0, 0);
  unsigned long long c0 = strtoull(argv[3], 0, 0), cnt = strtoull(argv[4], 0, 0);
  /* rocRAND's engine: key = (seed lo, seed hi); counter = (offset/4 as 64 bits, subsequence as 64 bits). */
  rocrand_device::philox4x32_10_engine e(seed, stream, 4ULL * c0);
  for (unsigned long long i = 0; i < 4 * cnt; ++i) printf("%u\n", e());
  return 0;
}
"""


@pytest.mark.skipif(not (os.path.exists(ROCRAND_HDR) and shutil.which("g++")),
                    reason="rocRAND headers or g++ not available")
@pytest.mark.parametrize("seed,stream,c0", [(0, 0, 0), (12345, 0, 77), (2**40 + 3, 1, 2**33 + 5),
                                            (0xDEADBEEFCAFEF00D, 2, 123456789)])
def test_philox_matches_independent_implementation(seed, stream, c0):
    """Cross-check against rocRAND's (independently written) header implementation."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(_PROG)
        subprocess.run(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", src, "-o", exe],
                       check=True, capture_output=True)
        cnt = 64
        out = subprocess.run([exe, str(seed), str(stream), str(c0), str(cnt)], check=True,
                             capture_output=True, text=True).stdout.split()
    ref = np.array([int(x) for x in out], dtype=np.uint64).reshape(cnt, 4)
    mine = philox.raw_words(seed, stream, np.arange(c0, c0 + cnt, dtype=np.uint64)).astype(np.uint64)
    assert np.array_equal(ref, mine)


def test_gaussian_statistics():
    z = philox.gaussian(7, 0, 400_000)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # no lag-1 correlation, and the cos/sin pair of one counter is uncorrelated
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5.0 / np.sqrt(n)
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5.0 / np.sqrt(n / 2)
    # fourth moment of N(0,1) is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_streams_and_seeds_differ():
    a = philox.gaussian(1, 0, 1000)
    b = philox.gaussian(1, 1, 1000)
    c = philox.gaussian(2, 0, 1000)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.2 and abs(np.corrcoef(a, c)[0, 1]) < 0.2
    assert np.array_equal(a, philox.gaussian(1, 0, 1000))
    # a window of the stream equals the same elements of the full stream
    assert np.array_equal(philox.gaussian(1, 0, 10, start=501), a[501:511])


def test_test_matrix_layout():
    n, r = 37, 5
    om = philox.test_matrix(3, n, r)
    flat = philox.gaussian(3, 0, n * r)
    for i, j in [(0, 0), (5, 0), (0, 1), (36, 4), (11, 3)]:
        assert om[i, j] == flat[j * n + i]
