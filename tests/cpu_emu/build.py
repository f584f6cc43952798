"""Build the CPU harness: the library sources (unchanged) compiled for the
host against include/hip/hip_runtime.h of this folder, with
AddressSanitizer and UndefinedBehaviorSanitizer, linked to driver.cpp.
TEST INFRASTRUCTURE: never loaded by the package."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRCS = [os.path.join(ROOT, "paper_2503_20605_amd", "csrc", f) for f in ("iblb.hip", "mlp.hip")]
OUT = os.path.join(HERE, "iblb_emu_driver")
CXX = "/opt/rocm/llvm/bin/clang++"


def sources():
    csrc = os.path.join(ROOT, "paper_2503_20605_amd", "csrc")
    return [os.path.join(csrc, f) for f in os.listdir(csrc)] + [
        os.path.join(HERE, "driver.cpp"), os.path.join(HERE, "include", "hip", "hip_runtime.h"),
        os.path.join(ROOT, "include", "iblb.h")]


def build(force=False, verbose=False):
    if (not force and os.path.exists(OUT)
            and os.path.getmtime(OUT) > max(os.path.getmtime(s) for s in sources())):
        return OUT
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2503_20605_amd", "csrc"),
           "-x", "c++"] + SRCS + [os.path.join(HERE, "driver.cpp"), "-o", OUT]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return OUT


if __name__ == "__main__":
    build(force=True, verbose=True)
