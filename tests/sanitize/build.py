"""Build the host sanitizer checks (CPU only, no GPU needed) into _build/:

  oracle_asan       the CPU oracle (oracle/hj_oracle.c) with its checks in
                    oracle_asan_main.c, gcc -fsanitize=address,undefined;
  hj_validate_asan  libhj's C ABI with hj_api.hip's host code built with the
                    address and undefined-behaviour sanitizers (device code as
                    usual), driven by hj_validate_main.cpp through every
                    argument-validation path.

    python tests/sanitize/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OBJ = os.path.join(ROOT, "_build")
CSRC = os.path.join(ROOT, "paper_2006_16465_amd", "csrc")
INC = os.path.join(ROOT, "include")
ORACLE_BIN = os.path.join(OBJ, "oracle_asan")
HJ_BIN = os.path.join(OBJ, "hj_validate_asan")
OTHER_OBJS = ["hj_kernels.o", "hj_refine.o", "hj_vc.o", "hj_batch.o", "hj_solve1d_wg.o"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False):
    os.makedirs(OBJ, exist_ok=True)
    _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
          os.path.join(ROOT, "oracle", "hj_oracle.c"), os.path.join(HERE, "oracle_asan_main.c"),
          "-lm", "-o", ORACLE_BIN], verbose)
    missing = [o for o in OTHER_OBJS if not os.path.exists(os.path.join(OBJ, o))]
    if missing:
        from paper_2006_16465_amd import build as hip_build
        hip_build.build(verbose=verbose, incremental=True)
    api_obj = os.path.join(OBJ, "hj_api_asan.o")
    # host-side sanitizers only (-Xarch_host before each flag); the device
    # code of hj_api.hip is built as in the library
    _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-fPIC",
          "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer", "-I", INC, "-I", CSRC,
          "-c", os.path.join(CSRC, "hj_api.hip"), "-o", api_obj], verbose)
    _run(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++20", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", "-I", INC, os.path.join(HERE, "hj_validate_main.cpp"), api_obj]
         + [os.path.join(OBJ, o) for o in OTHER_OBJS]
         + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", HJ_BIN], verbose)
    return ORACLE_BIN, HJ_BIN


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    build(verbose="-v" in sys.argv)
