"""Build liblyaf.so (the library) and libpeaks.so (the rate microbenchmarks
the benchmark reports against) for gfx950 with hipcc, in-tree next to this
file.  Beside each library a ``.srchash`` file records the SHA-256 of the
sources it was built from; the binding refuses a library whose sources have
changed since (content, not file times, which a copied tree may not keep)."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblyaf.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HEADERS = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [
    os.path.join(ROOT, "include", "lyaf.h")]
PEAKS_LIB = os.path.join(HERE, "libpeaks.so")
PEAKS_SOURCES = [os.path.join(HERE, "peaks", "lyaf_peaks.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep the compensated sums as written
    "-fno-fast-math", "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"),
]


def source_hash(paths=None) -> str:
    """SHA-256 over the library's sources and headers (names and contents)."""
    h = hashlib.sha256()
    for p in sorted(SOURCES + HEADERS if paths is None else paths):
        h.update(os.path.relpath(p, ROOT).encode())
        h.update(b"\0")
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def built_hash(lib: str = LIB):
    """The source hash recorded when ``lib`` was built, or None."""
    try:
        with open(lib + ".srchash") as f:
            return f.read().strip()
    except OSError:
        return None


def needs_build() -> bool:
    return not os.path.exists(LIB) or built_hash(LIB) != source_hash()


def _hipcc(out: str, sources, verbose: bool, deps=None) -> str:
    digest = source_hash(deps if deps is not None else list(sources))
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, out)
    with open(out + ".srchash", "w") as f:
        f.write(digest + "\n")
    return out


def build(verbose: bool = False) -> str:
    _hipcc(PEAKS_LIB, PEAKS_SOURCES, verbose,
           deps=PEAKS_SOURCES + [os.path.join(ROOT, "include", "lyaf_peaks.h")])
    return _hipcc(LIB, SOURCES, verbose, deps=SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
