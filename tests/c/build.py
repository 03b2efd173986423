"""Builds the C consumer of the ABI (tests/c/abi_solve.c) against the
in-tree library, with gcc: plain C, the HIP runtime's C API for device
memory, and the library's header."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2006_08498_amd")
EXE = os.path.join(HERE, "abi_solve")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "abi_solve.c"), "-o", EXE + ".tmp",
           "-L", PKG, "-lchase_mi355x", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2006_08498_amd",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
