"""Build the gfx950 engine library in-tree.

1. the process compiler writes csrc/gen/<process>.hip and process_table.inc;
2. hipcc compiles every generated kernel file and the runtime for gfx950,
   and each unit's device assembly is checked for half-spilled register
   pairs (isa_check.py), a miscompile that yields wrong values silently;
3. the objects are linked into libme_mi355x.so next to this file.

Run as ``python -m paper_2312_02898_amd.build`` (also called by the graft
entry point).  Every call compiles (objects of unchanged sources are reused).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libme_mi355x.so")

PROCESSES = ["eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg", "uutt", "uxutt",
             "uuttg", "uxuttg", "ugttu", "guttu", "uxgttux", "guxttux",
             "uuttgg", "uxuttgg", "ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux",
             "uuttuux", "uuttddx", "uuttuu", "udttud", "uxuxttuxux"]

HIPCC = os.environ.get("HIPCC", "hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (they have given silent wrong results on these parts)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # spill VGPRs to AGPRs before scratch memory
         "-mllvm", "-amdgpu-spill-vgpr-to-agpr=1",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# No fast-math flags.  -fno-signed-zeros -ffinite-math-only on the generated
# kernels let the compiler fold the products and sums with structurally zero
# components (x*0, x+0) and made them 10-30 % faster, but some schedules of
# four kernels (FP32 and FP64, whole-process and split parts) then gave
# wrong results that the same code without the flags does not give.


def _digest(paths, extra=""):
    h = hashlib.sha256(extra.encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src, deps):
    os.makedirs(OBJ, exist_ok=True)
    base = os.path.splitext(os.path.basename(src))[0]
    tag = _digest([src] + deps, " ".join(FLAGS))
    obj = os.path.join(OBJ, f"{base}-{tag}.o")
    if not os.path.exists(obj):
        tmp = obj + ".tmp"
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
        # the object is cached under the digest of its inputs: if any input
        # changed while it compiled, the object may hold other code than its
        # name says, and it is not kept
        if _digest([src] + deps, " ".join(FLAGS)) != tag:
            os.remove(tmp)
            raise RuntimeError(f"{src} or a header changed during its compile; build again")
        os.replace(tmp, obj)
    _check_device_code(src, obj)
    return obj


def _check_device_code(src, obj):
    """Compile the unit's device code to assembly once more and reject it if
    the compiler spilled half of a 64-bit register pair (isa_check): such a
    kernel computes wrong values with no fault.  The result is cached next
    to the object."""
    from . import isa_check
    stamp = obj + ".isa-ok"
    if os.path.exists(stamp):
        return
    asm = obj + ".s.tmp"
    cmd = [HIPCC] + FLAGS + ["-S", "--offload-device-only", src, "-o", asm]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed for {src}:\n{r.stderr[-4000:]}")
    with open(asm) as f:
        text = f.read()
    os.remove(asm)
    bad = isa_check.half_reloads(text)
    if bad:
        raise RuntimeError(f"{src}: the device compiler reloads half of a spilled 64-bit register pair "
                           f"(the kernel would compute wrong values); change the schedule:\n" + "\n".join(bad[:5]))
    with open(stamp, "w"):
        pass


def build(processes=None, jobs=None, verbose=True) -> str:
    """Generate, compile and link; builds of one tree run one at a time (a
    lock file), since they share csrc/gen and the object cache."""
    import fcntl
    os.makedirs(OBJ, exist_ok=True)
    with open(os.path.join(OBJ, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        return _build_locked(processes, jobs, verbose)


def _build_locked(processes, jobs, verbose) -> str:
    sys.path.insert(0, ROOT)
    from paper_2312_02898_amd.procgen import codegen
    procs = processes or PROCESSES
    srcs = codegen.generate(GEN, names=procs)
    hdrs = [os.path.join(CSRC, f) for f in ("helas.hpp", "kernels.hpp", "me_types.h", "colour_mfma.hpp", "split.hpp", "epilogue.hpp")]
    table = os.path.join(GEN, "process_table.inc")
    # a part kernel of a split process, <name>__<form>_<j>.hip, shares <name>_proc.inc
    units = [(s, hdrs + [os.path.join(GEN, os.path.basename(s)[:-4].split("__")[0] + "_proc.inc")])
             for s in srcs]
    units.append((os.path.join(CSRC, "runtime.cpp"), hdrs + [table, os.path.join(ROOT, "include", "me.h"),
                                                             os.path.join(CSRC, "channels.hpp"),
                                                             os.path.join(CSRC, "handle.hpp")]))
    hdrs = hdrs + [os.path.join(CSRC, "handle.hpp")]
    for extra in ("server.cpp", "unweight.cpp", "rambo.cpp", "channels.cpp", "noalloc.cpp"):
        units.append((os.path.join(CSRC, extra),
                      hdrs + [os.path.join(CSRC, "server_core.hpp"), os.path.join(CSRC, "channels.hpp"),
                              os.path.join(ROOT, "include", "me.h")]))
    jobs = jobs or min(len(units), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(*u), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    # drop stale objects
    keep = set(objs) | {o + ".isa-ok" for o in objs}
    for f in os.listdir(OBJ):
        p = os.path.join(OBJ, f)
        if p not in keep and (f.endswith(".o") or f.endswith(".isa-ok")):
            os.remove(p)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
