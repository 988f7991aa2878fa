"""Build the CPU oracle shared library (test infrastructure only).

Plain gcc, -O2, no fast-math: the oracle's arithmetic is IEEE FP64 as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rng.c", "sampler.c", "driver.c", "closed_form.c", "cv.c", "rhee_glynn.c"]
LIB = os.path.join(HERE, "liboracle.so")


SAN_LIB = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """liboracle.so; with sanitize, liboracle_san.so built with AddressSanitizer
    and UndefinedBehaviorSanitizer (CPU code; load it with the ASan runtime
    preloaded and ORACLE_LIB pointing at it)."""
    out = SAN_LIB if sanitize else LIB
    cmd = ["gcc", "-O1" if sanitize else "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter", "-fno-fast-math"]
    cmd += SAN_FLAGS if sanitize else []
    cmd += ["-o", out + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
