"""Builds libhx.so for gfx950 in-tree: one translation unit per polynomial degree and mesh topology
plus the host runtime, compiled in parallel with hipcc and linked into paper_2408_12479_amd/libhx.so."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhx.so")
DEGREES = range(1, 7)
# mesh topologies: lattice of trilinear cells, lattice with stored geometry, general mesh
TOPOLOGIES = range(3)

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + "\n".join(lines))
    return "\n".join(lines)


def build(jobs=None, verbose=False):
    """Compiles every translation unit and links libhx.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    units = []
    for p in DEGREES:
        for t in TOPOLOGIES:
            units.append(([hipcc] + FLAGS + [f"-DHX_DEGREE={p}", f"-DHX_TOPO={t}", "-c",
                                            os.path.join(CSRC, "hx_degree.hip"),
                           "-o", os.path.join(BUILD, f"hx_p{p}_t{t}.o")], f"p{p}/t{t}"))
    # the only matrix instructions of the library are the FP64 issue-rate probe's (hx_api.hip): its
    # accumulators stay in VGPRs instead of being copied to and from AGPRs in every loop iteration
    units.append(([hipcc] + FLAGS + ["-mllvm", "-amdgpu-mfma-vgpr-form", "-c", os.path.join(CSRC, "hx_api.hip"),
                   "-o", os.path.join(BUILD, "hx_api.o")], "api"))
    units.append(([hipcc] + FLAGS + ["-c", os.path.join(CSRC, "hx_solver.hip"),
                   "-o", os.path.join(BUILD, "hx_solver.o")], "solver"))
    units.append(([hipcc] + FLAGS + ["-c", os.path.join(CSRC, "hx_stability.hip"),
                   "-o", os.path.join(BUILD, "hx_stability.o")], "stability"))
    units.append(([hipcc] + FLAGS + ["-c", os.path.join(CSRC, "hx_mesh.hip"),
                   "-o", os.path.join(BUILD, "hx_mesh.o")], "mesh"))
    jobs = jobs or min(len(units), max(1, os.cpu_count() or 1), 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {ex.submit(_run, cmd): name for cmd, name in units}
        for f in cf.as_completed(futs):
            out = f.result()
            if verbose:
                print(f"[build] {futs[f]} done", flush=True)
                if out.strip():
                    print(out)
    objs = [os.path.join(BUILD, f"hx_p{p}_t{t}.o") for p in DEGREES for t in TOPOLOGIES] + [
        os.path.join(BUILD, n) for n in ("hx_api.o", "hx_solver.o", "hx_stability.o", "hx_mesh.o")]
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lrocsolver", "-lrocblas"])
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] linked {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
