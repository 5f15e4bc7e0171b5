"""Address and undefined-behaviour sanitizer runs of host code on the CPU.

* The library's layout planner (hl_layout.cpp: validation, site orders, pull
  tables, int16 deltas, link data, schedules, the XCD map, the coupling
  construction) built with g++ -fsanitize=address,undefined together with
  tests/sanitize/layout_check.cpp, which plans every site order and schedule
  for a few geometries and runs the planner's exhaustive layout check on each.
* The FP64 oracle built with the same sanitizers and loaded into a child
  Python (libasan preloaded) that runs a set of pins covering every part of
  its step (moments, collision, streaming with every boundary rule, iolet
  means, coupling, wall shear stress, Eq. (2)).
No GPU code is built here.
"""
import os
import shutil
import struct
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_04144_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _write_domains(path, geos):
    with open(path, "wb") as fh:
        fh.write(struct.pack("<i", len(geos)))
        for g in geos:
            n = g.n
            fh.write(struct.pack("<qi", n, len(g.iolets)))
            fh.write(np.ascontiguousarray(g.coords, np.int32).tobytes())
            fh.write(np.ascontiguousarray(g.nbr, np.int32).tobytes())
            fh.write(struct.pack("<q", g.q.size))
            fh.write(np.ascontiguousarray(g.q_site, np.int64).tobytes())
            fh.write(np.ascontiguousarray(g.q_dir, np.int8).tobytes())
            fh.write(np.ascontiguousarray(g.q, np.float32).tobytes())
            for io in g.iolets:
                fh.write(struct.pack("<i", 0 if io.kind == "inlet" else 1))
                fh.write(np.asarray(io.centre, np.float64).tobytes())
                fh.write(np.asarray(io.normal, np.float64).tobytes())
                fh.write(struct.pack("<d", float(io.radius)))


def test_layout_planner_under_sanitizers():
    tree = synth.tree_geometry(3, 7.0, 20100416, lam=6.0)
    cases = {
        "cylinder": [synth.cylinder(nz=24, q="random", seed=2)],
        "tree": [tree],
        "periodic_ragged": [synth.cylinder(nx=9, ny=9, nz=7, radius=3.3, ends="periodic")],
        "coupled": [synth.tubes(1, radius=4.0, length=12), synth.tubes(3, radius=4.0, length=12)],
        "tree_pair": [synth.tree_geometry(2, 6.0, 7, lam=6.0),
                      synth.tree_geometry(2, 6.0, 7, lam=6.0, radius_scale=1.5, mirror=True, venous=True)],
        # random porous blocks: isolated sites, one-voxel channels, sites walled on most links,
        # bricks that are nearly empty; closed and periodic in x
        "porous": [synth.box(21, 19, 23, periodic=(False, False, False),
                             solid=np.random.default_rng(5).random((23, 19, 21)) < 0.35).with_q("random", seed=6),
                   synth.box(34, 9, 11, periodic=(True, False, False),
                             solid=np.random.default_rng(8).random((11, 9, 34)) < 0.25).with_q("random", seed=9)],
    }
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "layout_check")
        cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, "hl_layout.cpp"), os.path.join(ROOT, "tests", "sanitize", "layout_check.cpp"),
               "-o", exe]
        subprocess.run(cmd, check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        for name, geos in cases.items():
            path = os.path.join(tmp, name + ".bin")
            _write_domains(path, geos)
            p = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=600)
            assert p.returncode == 0, (name, p.stdout[-3000:], p.stderr[-3000:])
            assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, (name, p.stderr[-3000:])
            assert "plans checked" in p.stdout, (name, p.stdout)


PIN_SUBSET = ("rest_state or mass_budget or sparse_addressing or at_half or second_node or waveform or "
              "velocity_factors or reverse_reading or feq or collision or wall_shear or momentum_budget or "
              "exchange_directions or state_injection or from_outside")


def test_oracle_under_sanitizers():
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("libasan not found")
    from oracle import build as ob
    with tempfile.TemporaryDirectory() as tmp:
        lib = ob.build(out=os.path.join(tmp, "oracle_san.so"), extra=SAN)
        env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0", ORACLE_LIB_OVERRIDE=lib,
                   OMP_NUM_THREADS="2")
        p = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-p", "no:cacheprovider",
                            "-m", "not gpu", "-k", PIN_SUBSET], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=900)
        assert p.returncode == 0, (p.stdout[-3000:], p.stderr[-3000:])
        assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-3000:]
        assert " passed" in p.stdout
