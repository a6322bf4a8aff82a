"""The stiffness product's walk over its mode records, compiled on the host.

The product gathers its modes in chunks of a compile-time record count (a
full chunk of KC records, one chunk of KC / 2, chunks of 4); every chunk must
stay inside the gp records staged in LDS (gp = g rounded up to 4).  A walk
that ran past gp read records that were never staged and gave results that
changed from run to run; the kernels now check the walk at compile time
(static_assert on chunk_walk_exact) for their own KC.  This test runs the
same header on the host for every chunk size the in-flight settings can
give, and rebuilds each walk from its chunks.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_06841_amd", "csrc")
GPMAX = 64  # QP_MAX_MODES, already a multiple of 4

PROGRAM = r"""
#include <cstdio>
#include "qp_chunk_walk.h"
int main() {
    for (int KC = 4; KC <= 64; KC += 4)
        for (int gp = 4; gp <= %d; gp += 4) {
            std::printf("%%d %%d %%d %%d", KC, gp, qp::chunk_walk_end(KC, gp),
                        (int)qp::chunk_walk_exact(KC, gp));
            // the chunks, as the kernels take them
            int rb = 0;
            for (; rb + KC <= gp; rb += KC) std::printf(" %%d:%%d", rb, KC);
            if (qp::take_half_chunk(KC, rb, gp)) { std::printf(" %%d:%%d", rb, KC / 2); rb += KC / 2; }
            for (; rb < gp; rb += 4) std::printf(" %%d:4", rb);
            std::printf("\n");
        }
    return 0;
}
""" % GPMAX


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
        KC, gp, end, exact = map(int, f[:4])
        chunks = [tuple(map(int, c.split(":"))) for c in f[4:]]
        table[(KC, gp)] = (end, exact, chunks)
    return table


def test_every_walk_covers_the_staged_records_exactly(walks):
    for (KC, gp), (end, exact, chunks) in walks.items():
        assert end == gp, (KC, gp, chunks)
        pos = 0
        for start, size in chunks:
            assert start == pos and start % 4 == 0 and size in (KC, KC // 2, 4), (KC, gp, chunks)
            assert start + size <= gp, (KC, gp, chunks)
            pos += size
        assert pos == gp, (KC, gp, chunks)


def test_exact_for_every_in_flight_setting(walks):
    # the plane-tile product: KC = (inflight / KR) rounded down to a multiple
    # of 4 when that is at least 8, else 4; the generic product: KC = inflight
    for inflight in range(4, 65, 4):
        for KR in (1, 2, 3):
            q = inflight // KR
            KC = (q // 4) * 4 if q >= 8 else 4
            assert walks[(KC, GPMAX)][1] == 1, (inflight, KR, KC)
        assert walks[(inflight, GPMAX)][1] == 1, inflight


def test_half_chunk_case_that_once_ran_past_the_records(walks):
    # 24 gathers in flight over two right-hand sides: KC = 12; with the 17
    # modes of the headline problem gp = 20.  A 6-record half chunk at 12
    # would leave the 4-chunks starting at 18 and reading records 20 and 21.
    end, exact, chunks = walks[(12, 20)]
    assert chunks == [(0, 12), (12, 4), (16, 4)] and end == 20
