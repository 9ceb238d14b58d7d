"""Build the HIP library ``librz.so`` for gfx950 with hipcc (in-tree).

Usage: python -m paper_2211_14284_amd.build   (or call build())
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librz.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["tables1d.cpp", "patch.cpp", "geom.cpp", "vec_local.cpp", "hmg.cpp", "rz_api.cpp", "k_grad.hip", "k_grad_pd.hip", "k_common.hip",
           "k_quad.hip", "k_quad_mfma.hip", "k_vec.hip", "k_vec_relax.hip", "mlp.hip", "k_hmg.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _pass_tables():
    """Run gen_pass_tables (host g++) to write the compile-time patch schedules."""
    exe = os.path.join(BUILD, "gen_pass_tables")
    cmd = [os.environ.get("CXX", "g++"), "-O1", "-std=c++17", "-I", CSRC, os.path.join(CSRC, "gen_pass_tables.cpp"),
           os.path.join(CSRC, "patch.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    r = subprocess.run([exe, os.path.join(BUILD, "pass_tables.inc")], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gen_pass_tables failed\n{r.stdout}\n{r.stderr}")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-I", BUILD, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    _pass_tables()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
