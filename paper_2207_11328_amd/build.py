"""Build libsph.so (hand-written HIP for gfx950) in-tree with hipcc.

    python -m paper_2207_11328_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsph.so")
# (source, object, extra defines): the pair loops are compiled once per
# smoothing kernel so the instances of the four kernels build in parallel
PAIR_SOURCES = ["forces_pairs.hip", "forces_backward_pairs.hip"]
SOURCES = ([(s, s.replace(".hip", ".o"), []) for s in
            ["neighbors.hip", "forces.hip", "forces_backward.hip", "integrate.hip", "probe.hip"]] +
           [(s, s.replace(".hip", "_k%d.o" % k), ["-DSPH_KERNEL_KIND=%d" % k]) for s in PAIR_SOURCES for k in range(4)])
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def flags() -> list:
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++20", "-fPIC",
        # packed FP32 instructions are disabled for correctness on this target
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + INCLUDE, "-I" + CSRC,
        "-Wall", "-Wno-unused-function",
        # per-kernel register, scratch and LDS usage, checked below
        "-Rpass-analysis=kernel-resource-usage",
    ]


class ScratchError(RuntimeError):
    pass


def resource_usage(text: str) -> dict:
    """{kernel: {field: value}} from the compiler's kernel-resource-usage
    remarks (function name, registers, scratch, spills, dynamic stack)."""
    out, cur = {}, None
    for ln in text.splitlines():
        if "[-Rpass-analysis=kernel-resource-usage]" not in ln or "remark:" not in ln:
            continue
        body = ln.split("remark:", 1)[1].replace("[-Rpass-analysis=kernel-resource-usage]", "").strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            out[cur][k.strip()] = v.strip()
    return out


def check_no_scratch(src: str, usage: dict):
    """Fail the build if any kernel of `src` uses scratch memory: vector
    register spills or a stack would turn the pair loops' register traffic
    into memory traffic.  (Scalar register spills go to vector register
    lanes, not to memory, and are allowed.)"""
    bad = []
    for fn, u in usage.items():
        scratch = int(u.get("ScratchSize [bytes/lane]", "0"))
        spills = int(u.get("VGPRs Spill", "0"))
        dyn = u.get("Dynamic Stack", "False") != "False"
        if scratch or spills or dyn:
            bad.append("%s: scratch %d B/lane, VGPR spills %d, dynamic stack %s" % (fn, scratch, spills, dyn))
    if bad:
        raise ScratchError("kernels of %s use scratch memory:\n  %s" % (src, "\n  ".join(bad)))


def build(verbose: bool = False, jobs: int = 0) -> str:
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    procs = []
    objs = []
    for src, oname, defs in SOURCES:
        obj = os.path.join(objdir, oname)
        cmd = [cc] + flags() + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
    usage = resource_usage(text)
    check_no_scratch(src, usage)
    # the host pass does not know the packed-fp32 target feature: harmless;
    # the resource remarks were checked above; the source-line echo of a
    # remark is a line of code with a caret line under it
    lines = []
    skip = 0
    for ln in text.splitlines():
        if skip:
            skip -= 1
            continue
        if "kernel-resource-usage" in ln:
            skip = 2 if "Function Name" in ln else 0
            continue
        if "packed-fp32-ops" in ln or not ln.strip():
            continue
        lines.append(ln)
    if lines:
        print("\n".join(lines), file=sys.stderr)
    return usage


if __name__ == "__main__":
    print(build(verbose=True))
