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
# Second build whose host-side chunking ignores the box budget (plain runs
# of the chunk size), so that spreading chunks overflow the kernel's LDS box
# and take its direct-atomic path.
OUT_DIRECT = os.path.join(HERE, "iblb_emu_driver_direct")
CXX = "/opt/rocm/llvm/bin/clang++"


def sources():
    csrc = os.path.join(ROOT, "paper_2503_20605_amd", "csrc")
    return [os.path.join(csrc, f) for f in os.listdir(csrc)] + [
        os.path.join(HERE, "driver.cpp"), os.path.join(HERE, "include", "hip", "hip_runtime.h"),
        os.path.join(ROOT, "include", "iblb.h")]


def build(force=False, verbose=False, direct=False):
    out = OUT_DIRECT if direct else OUT
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) > max(os.path.getmtime(s) for s in sources())):
        return out
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2503_20605_amd", "csrc")]
    if direct:
        cmd += ["-DIBLB_CHUNK_BUDGET=1000000000"]
    cmd += ["-x", "c++"] + SRCS + [os.path.join(HERE, "driver.cpp"), "-o", out]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(force=True, verbose=True)
    build(force=True, verbose=True, direct=True)
