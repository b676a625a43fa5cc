"""Build the test-only HIP kernels of tests/native (fp64 division and square
root) with the library's compiler flags into tests/native/libfp64ops.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libfp64ops.so")


def build(verbose: bool = False) -> str:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2008_13461_amd import build as B
    cmd = [B.HIPCC, *B.FLAGS, "-shared", "-o", LIB + ".tmp", os.path.join(HERE, "fp64_ops.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
