"""Builds libpn.so (the HIP C-ABI library) in-tree for gfx950 with hipcc.

Each source is compiled to an object in parallel (one translation unit per
stencil order), then linked into paper_1807_00410_amd/libpn.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpn.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++20", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result", "-fconstexpr-steps=200000000",
]

SOURCES = ["pn_api.hip", "pn_batch.hip", "pn_nn.hip"] + ["pn_order_%d.hip" % n for n in range(1, 8)]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed (%d): %s" % (r.returncode, " ".join(cmd[-3:])))


def _newest_input(path, seen=None):
    """Newest modification time of a source and of the project headers it
    includes (quoted #include lines, followed recursively)."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return 0.0
    seen.add(path)
    t = os.path.getmtime(path)
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#include") and '"' in line:
                name = line.split('"')[1]
                for d in (os.path.dirname(path), os.path.join(ROOT, "include")):
                    t = max(t, _newest_input(os.path.normpath(os.path.join(d, name)), seen))
    return t


def build(verbose=False, jobs=None, incremental=False):
    """Compiles every source (incremental=True: only objects older than their
    source or any header) and links libpn.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= _newest_input(os.path.join(HERE, "csrc", src)):
            continue
        cmds.append([hipcc] + HIPCC_FLAGS + inc + ["-c", os.path.join(HERE, "csrc", src), "-o", obj])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
