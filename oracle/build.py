"""Build the FP64 CPU oracle (test infrastructure) into oracle/libsasa_oracle.so.

Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sasa_oracle.cc")
SOURCES = [SRC, os.path.join(HERE, "predicates.cc"), os.path.join(HERE, "volume_oracle.cc"),
           os.path.join(HERE, "curvature_oracle.cc")]
HEADERS = [os.path.join(HERE, "sasa_oracle.h"), os.path.join(HERE, "predicates.h")]
LIB = os.path.join(HERE, "libsasa_oracle.so")


def build(force=True, march_native=False):
    """Compile the oracle with g++: -O3 for x86-64-v3 (AVX2/FMA, which every
    host of this work has; the built library travels with the tree, so not
    -march=native unless asked).  No fast-math and no contraction into fused
    operations: the predicates' error bounds assume separately rounded ones."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in SOURCES):
        return LIB
    flags = ["-O3", "-std=c++17", "-shared", "-fPIC", "-fno-fast-math", "-ffp-contract=off"]
    flags.append("-march=native" if march_native else "-march=x86-64-v3")
    tmp = LIB + ".tmp"
    cmd = ["g++", *flags, *SOURCES, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(HERE, "libsasa_oracle_san.so")


def build_sanitized():
    """The same sources with AddressSanitizer and UndefinedBehaviorSanitizer
    (-O1, frame pointers, every undefined-behaviour report fatal) into
    oracle/libsasa_oracle_san.so, for runs in a process that preloads the
    sanitizer runtime (tests/test_oracle_sanitizers.py)."""
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-std=c++17", "-shared", "-fPIC", "-fno-fast-math", "-ffp-contract=off"]
    tmp = SAN_LIB + ".tmp"
    subprocess.run(["g++", *flags, *SOURCES, "-o", tmp], check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build(force=True, march_native="--native" in sys.argv))
