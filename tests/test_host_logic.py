"""Host-side logic of the library checked on the CPU (no GPU needed)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_2698_amd", "csrc")

HILBERT_CHECK = r"""
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "hilbert.hpp"
template <int B> int check() {
    const int n = 1 << B;
    std::vector<std::pair<uint32_t, int>> v;
    for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y)
            for (int z = 0; z < n; ++z) v.push_back({tds::hilbert3<B>(x, y, z), (x << 20) | (y << 10) | z});
    std::sort(v.begin(), v.end());
    int bad = 0;
    for (size_t i = 0; i < v.size(); ++i) bad += v[i].first != i;            // a bijection onto [0, n^3)
    for (size_t i = 1; i < v.size(); ++i) {                                 // unit steps
        const int a = v[i - 1].second, b = v[i].second;
        bad += std::abs((a >> 20) - (b >> 20)) + std::abs(((a >> 10) & 1023) - ((b >> 10) & 1023)) +
               std::abs((a & 1023) - (b & 1023)) != 1;
    }
    std::printf("B=%d bad=%d\n", B, bad);
    return bad;
}
int main() { return check<1>() + check<2>() + check<3>() + check<5>() + check<6>(); }
"""


def test_hilbert_index_is_a_hilbert_curve(tmp_path):
    """The spatial layout's cell order visits every cell once, moving to an
    adjacent cell at each step (the defining property of a Hilbert curve)."""
    src = tmp_path / "hilbert_check.hip"
    src.write_text(HILBERT_CHECK)
    exe = tmp_path / "hilbert_check"
    try:
        subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                       check=True, capture_output=True)
    except FileNotFoundError:
        pytest.skip("hipcc not available")
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
