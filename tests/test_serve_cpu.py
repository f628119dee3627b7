"""Host logic of the serving loop that needs no GPU: the first-fit
allocator that admits requests into the device arena (compiled with g++
against the library's own header and checked against a byte-map model), and
the request bookkeeping of the Python driver."""

import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def arena_driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_driver")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I",
                           os.path.join(ROOT, "paper_2010_14058_amd", "csrc"),
                           os.path.join(HERE, "arena_driver.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_arena_against_model(arena_driver, seed):
    out = subprocess.run([arena_driver, str(seed)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


def test_request_sizes():
    from paper_2010_14058_amd import serve as S
    from tg_synth import graphs as G

    g = G.random_small_graph(12, 0.4, 3, 1)
    r = S.Request(0, g.row_ptr, g.col, g.types, g.L)
    assert r.n == g.n and r.m == g.m and r.status == -1
