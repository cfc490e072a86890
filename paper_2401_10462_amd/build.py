"""Build the HIP library (gfx950) into paper_2401_10462_amd/libsasa_hip.so."""
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libsasa_hip.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "volume.hip", "sorted_extract.hip", "incremental.hip", "api.hip")]
HEADERS = [os.path.join(CSRC, "sasa_internal.h"), os.path.join(CSRC, "exact_side.h"), os.path.join(INCLUDE, "sasa.h")]
# SHA-256 of the sources and flags the library was built from (written beside it)
HASH = LIB + ".srchash"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-mcode-object-version=5",
    # packed FP32 instructions stay off (hipcc pass-through to the device compiler)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
]


def source_hash():
    """Digest of every source and header and of the compiler flags."""
    h = hashlib.sha256()
    for p in SOURCES + HEADERS:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(f for f in FLAGS if not os.path.isabs(f)).encode())  # (the tree may move)
    return h.hexdigest()


def stale():
    """True if the library is missing or was built from other sources."""
    if not os.path.exists(LIB) or not os.path.exists(HASH):
        return True
    with open(HASH) as f:
        return f.read().strip() != source_hash()


def build(force=True, verbose=False):
    """Compile the library; always recompiles when force is set."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    with open(HASH, "w") as f:
        f.write(source_hash() + "\n")
    return LIB


if __name__ == "__main__":
    print(build(force=True))
