"""Build libhjpd.so for gfx950 with hipcc (in-tree).

Translation units are compiled in parallel: the C-ABI layer, the
linear-tanh unit and one kernel-instantiation unit per (family shape,
dtype).  All device code is compiled with packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libhjpd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# (lookup suffix, family type, real type)
INSTANCES = [
    ("cnorm2_f32", "CNorm<2>", "float"), ("cnorm2_f64", "CNorm<2>", "double"),
    ("cnorm3_f32", "CNorm<3>", "float"), ("cnorm3_f64", "CNorm<3>", "double"),
    ("cnorm4_f32", "CNorm<4>", "float"), ("cnorm4_f64", "CNorm<4>", "double"),
    ("cnorm10_f32", "CNorm<10>", "float"), ("cnorm10_f64", "CNorm<10>", "double"),
    ("quad_f32", "Quad", "float"), ("quad_f64", "Quad", "double"),
    ("pursuit_f32", "Pursuit", "float"), ("pursuit_f64", "Pursuit", "double"),
    ("isaacs_f32", "Isaacs", "float"), ("isaacs_f64", "Isaacs", "double"),
]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops' is not a recognized feature" not in l
                    and "is not a recognized feature for this target" not in l)
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    return err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every unit and link libhjpd.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    cmds, objs = [], []
    for name, fam, real in INSTANCES:
        o = os.path.join(BUILD, "inst_%s.o" % name)
        cmds.append([HIPCC, *FLAGS, "-DHJPD_FAM=%s" % fam, "-DHJPD_REAL=%s" % real, "-DHJPD_NAME=%s" % name,
                     "-c", os.path.join(CSRC, "hjpd_inst.hip"), "-o", o])
        objs.append(o)
    for unit in ("hjpd_api", "hjpd_lintanh", "hjpd_calib"):
        o = os.path.join(BUILD, unit + ".o")
        cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, unit + ".hip"), "-o", o])
        objs.append(o)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for msg in ex.map(_run, cmds):
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
