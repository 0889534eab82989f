"""Build step of the HIP library (hipcc, gfx950) into paper_2511_21264_amd/_lib/libmppi.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libmppi.so")
SOURCES = ["csrc/kernels.hip", "csrc/api.hip", "csrc/serve.hip", "csrc/qp.hip", "csrc/cov.hip", "csrc/episode.hip"]
HEADERS = ["csrc/devmodel.h", "csrc/philox.h", "csrc/dynamics.h", "csrc/collision.h", "csrc/step.h",
           "csrc/cost.h", "csrc/team.h", "csrc/kernels.h", "csrc/internal.h", "csrc/sched.h", "csrc/episode.h",
           "../include/mppi.h"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_*_f32) in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 division and square root from the hardware reciprocal / square
    # root (about 1 ulp) instead of the correctly rounded sequences: these
    # sit on the per-step dependency chains (Cholesky pivots, distances)
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    # multiply-adds fused only where one expression writes a * b + c: the
    # rounding of a formula then does not depend on the code it is inlined
    # into, which keeps the team, wave and split mappings bit-identical
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument", "-pthread",
]


def build(verbose=False, extra=()):
    os.makedirs(LIB_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + list(extra) + [os.path.join(HERE, s) for s in SOURCES] + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH
