"""The host plan is the same whatever the number of host threads that build it:
every field of plans built on 2, 3 and 8 threads equals the one-thread plan, on
meshes with and without subdomain labels (recursive bisection), overlap 1 and 2,
both interpolations, and a 32^3 mesh large enough that every phase splits its
work across the threads. Host logic only (g++ build of the plan source)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2606_20496_amd import meshgen as mg

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2606_20496_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("plan_threads") / "plan_threads")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC, os.path.join(HERE, "plan_threads_main.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def _write(d, m, *, labels=True, overlap=1, interp=0):
    os.makedirs(d, exist_ok=True)
    np.ascontiguousarray(m.xyz, dtype=np.float64).tofile(os.path.join(d, "xyz.bin"))
    np.ascontiguousarray(m.e2v, dtype=np.int32).tofile(os.path.join(d, "e2v.bin"))
    np.ascontiguousarray(m.dirichlet, dtype=np.uint8).tofile(os.path.join(d, "dir.bin"))
    if labels:
        np.ascontiguousarray(m.part, dtype=np.int32).tofile(os.path.join(d, "part.bin"))
    np.array([m.n_part, *m.boxes, overlap, interp], dtype=np.int32).tofile(os.path.join(d, "meta.bin"))


def _ragged():
    return mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))


CASES = {
    "cube8": (mg.small_cube, {}),
    "ragged": (_ragged, {}),
    "ragged_rcb": (_ragged, dict(labels=False)),
    "ragged_overlap2": (_ragged, dict(overlap=2)),
    "ragged_standard": (_ragged, dict(interp=1)),
    "reoriented": (lambda: mg.reorient(_ragged(), 7), {}),
    "stretched": (lambda: mg.box_mesh(16, 25, block=8, boxes=(2, 2, 2), faces=("z1",), zstretch=(1.1, 20.0)), {}),
    "annulus32": (lambda: mg.annulus_mesh(32, 3, block=8, boxes=(4, 4, 4)), {}),
    "annulus32_rcb_standard": (lambda: mg.annulus_mesh(32, 3, block=8, boxes=(4, 4, 4)), dict(labels=False, interp=1)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_plan_independent_of_thread_count(name, checker, tmp_path):
    make, kw = CASES[name]
    d = str(tmp_path / name)
    _write(d, make(), **kw)
    r = subprocess.run([checker, d, "2", "3", "8"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.split() == ["same", "2", "same", "3", "same", "8"]
