"""Build libmcsvt.so (HIP, gfx950) in-tree.

    python -m paper_1810_06860_amd.build [--jobs N] [--debug]

Compiles every csrc/*.hip to an object under _build/ and links them into
paper_1810_06860_amd/libmcsvt.so.  Always recompiles (the build is the
"does it compile" check), in parallel.
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmcsvt.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags(debug=False):
    return [f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
            "-O1" if debug else "-O3", f"-I{INCLUDE}", f"-I{CSRC}",
            # packed FP32 instructions stay off (they have given silent wrong
            # results on this hardware)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip"))


def _compile(src, flags):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc()] + flags + ["-c", src, "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (proc.stdout + proc.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    return src, obj, proc.returncode, out


def build(jobs=None, debug=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    flags = common_flags(debug)
    srcs = sources()
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    objs, failed = [], []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, rc, out in ex.map(lambda s: _compile(s, flags), srcs):
            if out.strip() and (verbose or rc):
                sys.stderr.write(out + "\n")
            if rc:
                failed.append(src)
            objs.append(obj)
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.debug, a.verbose))


if __name__ == "__main__":
    main()
