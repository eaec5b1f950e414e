"""Build librmdec.so (HIP, gfx950) in-tree.

Each translation unit is compiled to an object in parallel, then linked into
``paper_2108_12550_amd/librmdec.so``.  Usage: ``python -m paper_2108_12550_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librmdec.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # same float evaluation order as written: no contraction into FMA
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
SOURCES = ["rmdec_inst_t.hip", "rmdec_inst_o.hip", "rmdec_inst_q.hip", "rmdec_inst_l.hip", "rmdec_inst_p.hip",
           "rmdec_inst_k.hip", "rmdec_inst_n.hip", "rmdec_inst_m.hip", "rmdec_inst_g.hip", "rmdec_inst_h.hip",
           "rmdec_inst_j.hip", "rmdec_inst_i.hip", "rmdec_inst_f.hip", "rmdec_inst_e.hip", "rmdec_serve_l8.hip",
           "rmdec_serve_l4.hip", "rmdec_serve_l1.hip", "rmdec_mixed.hip", "rmdec_inst_a.hip", "rmdec_inst_b.hip",
           "rmdec_inst_c.hip", "rmdec_inst_d.hip", "rmdec_inst_r.hip", "rmdec_inst_s.hip", "rmdec_host.hip",
           "rmdec_serve.hip", "rmdec_fresh.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(line for line in p.stderr.splitlines() if noise not in line)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
