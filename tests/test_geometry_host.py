"""The GPU path's geometry code, compiled for the host, against the oracle.

csrc/geometry.hpp (incremental Siddon traversal for rows of A, closed-form
voxel chords for rows of A^T) is built with g++ and every entry it produces
is compared with the FP64 oracle (Siddon crossing merge / slab clipping).
This pins the device geometry on the CPU before any kernel runs."""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "geometry_host.cpp")
REC = np.dtype([("r", np.int32), ("c", np.int32), ("v", np.float64)])


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("geo") / "geometry_host")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-D__host__=", "-D__device__=",
                           "-D__forceinline__=inline", SRC, "-o", exe, "-lm"])
    return exe


def run(prog, mode, N, M, C, tmp_path):
    out = str(tmp_path / f"{mode}.bin")
    subprocess.check_call([prog, mode, str(N), str(M), str(C), out])
    d = np.fromfile(out, dtype=REC)
    shape = (M * C, N * N) if mode == "ray" else (N * N, M * C)
    m = sp.coo_matrix((d["v"], (d["r"], d["c"])), shape=shape).tocsr()
    assert m.nnz == len(d), "duplicate entries"
    return m


GEOMS = [(4, 4, 4), (16, 12, 16), (15, 9, 15), (37, 23, 41), (24, 10, 23), (8, 6, 7), (64, 90, 64),
         (128, 180, 128), (5, 7, 6), (64, 1, 64)]


@pytest.mark.parametrize("N,M,C", GEOMS)
def test_device_siddon_matches_oracle(prog, tmp_path, N, M, C):
    got = run(prog, "ray", N, M, C, tmp_path)
    ref = oracle.build_A(N, M, C)
    assert got.nnz == ref.nnz
    d = abs(got - ref)
    assert d.max() <= 1e-12


@pytest.mark.parametrize("N,M,C", GEOMS)
def test_device_voxel_chords_match_oracle(prog, tmp_path, N, M, C):
    got = run(prog, "voxel", N, M, C, tmp_path)
    ref = oracle.build_AT(N, M, C)
    assert got.nnz == ref.nnz
    d = abs(got - ref)
    assert d.max() <= 1e-12
