"""The stiffness product's walk over its mode records, compiled on the host.

The product gathers its g modes in chunks of a compile-time record count (full
chunks of KC records, one chunk of KC / 2, chunks of 4, then one chunk of the
1 to 3 records left).  Only the first g records are real: the staged records
past g are zero-weight padding up to a multiple of 4, and a walk that ran past
the staged records once read records that were never written and gave results
that changed from run to run.  This test runs the kernels' own walk
(`walk_records` in qp_chunk_walk.h) on the host for every chunk size the
in-flight settings can give and every mode count, and rebuilds each walk from
its chunks.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_06841_amd", "csrc")
GMAX = 64  # QP_MAX_MODES

PROGRAM = r"""
#include <cstdio>
#include <utility>
#include "qp_chunk_walk.h"
template <int KC> void walks() {
    for (int g = 0; g <= %d; ++g) {
        std::printf("%%d %%d", KC, g);
        qp::walk_records<KC>(g, [](auto Cc, int rb) {
            std::printf(" %%d:%%d", rb, (int)decltype(Cc)::value);
        });
        std::printf("\n");
    }
}
template <int... I> void all(std::integer_sequence<int, I...>) { (walks<4 * (I + 1)>(), ...); }
int main() { all(std::make_integer_sequence<int, 16>()); return 0; }
""" % GMAX


@pytest.fixture(scope="module")
def walks(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("walk")
    src = d / "walk.cpp"
    src.write_text(PROGRAM)
    exe = d / "walk"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        f = line.split()
        KC, g = int(f[0]), int(f[1])
        table[(KC, g)] = [tuple(map(int, c.split(":"))) for c in f[2:]]
    return table


def test_every_walk_covers_the_real_records_exactly(walks):
    assert len(walks) == 16 * (GMAX + 1)
    for (KC, g), chunks in walks.items():
        pos = 0
        for start, size in chunks:
            assert start == pos and size in (KC, KC // 2, 4, 3, 2, 1), (KC, g, chunks)
            assert start + size <= g, (KC, g, chunks)
            pos += size
        assert pos == g, (KC, g, chunks)
        # at most one chunk of fewer than 4 records, and only at the end
        assert all(s >= 4 for _, s in chunks[:-1]), (KC, g, chunks)


def test_in_flight_settings(walks):
    # the plane-tile product: KC = (inflight / KR) rounded down to a multiple
    # of 4 when that is at least 8, else 4; the generic product: KC = inflight
    for inflight in range(4, 65, 4):
        for KR in (1, 2, 3):
            q = inflight // KR
            KC = (q // 4) * 4 if q >= 8 else 4
            assert (KC, GMAX) in walks, (inflight, KR, KC)


def test_the_headline_and_icosahedral_walks(walks):
    # 17 modes (the eightfold field with eight mode pairs): two right-hand
    # sides keep KC = 8; the last chunk is the one real record past 16
    assert walks[(8, 17)] == [(0, 8), (8, 8), (16, 1)]
    # 13 icosahedral modes with KC = 8 (FP64, one right-hand side) and 16
    assert walks[(8, 13)] == [(0, 8), (8, 4), (12, 1)]
    assert walks[(16, 13)] == [(0, 8), (8, 4), (12, 1)]
    # 24 gathers in flight over two right-hand sides: KC = 12, and a half
    # chunk of 6 is now allowed, since no later chunk has to end at a
    # multiple of 4
    assert walks[(12, 17)] == [(0, 12), (12, 4), (16, 1)]
    assert walks[(12, 20)] == [(0, 12), (12, 6), (18, 2)]
