"""Build libintergrams.so for gfx950 with hipcc (in-tree)."""
import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libintergrams.so")
ARCH = os.environ.get("IG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=%s" % ARCH,
    # packed-FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


SAN_SO = os.path.join(HERE, "libintergrams_san.so")
# host code only: AddressSanitizer and UndefinedBehaviorSanitizer on the CPU side of the library
# (the device code is built as usual)
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-fno-omit-frame-pointer", "-g"]


def build(verbose=False, jobs=8, sanitize=False):
    """Compile every .hip source to an object and link the shared library (with sanitize: the
    host-sanitized variant libintergrams_san.so, for runs with the sanitizer runtime preloaded)."""
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    t0 = time.time()
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc"] + HIPCC_FLAGS + (SAN_FLAGS if sanitize else []) + ["-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            time.sleep(0.05)
    failed = False
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write("compile failed: %s\n%s\n" % (src, out))
        elif verbose and out.strip():
            sys.stderr.write(out + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    out = SAN_SO if sanitize else SO
    tmp = out + ".tmp%d" % os.getpid()
    link = ["hipcc", "-shared", "-fPIC", "--offload-arch=%s" % ARCH] + (SAN_FLAGS if sanitize else []) + objs + \
        ["-o", tmp, "-lpthread"]
    subprocess.check_call(link)
    os.replace(tmp, out)
    if verbose:
        sys.stderr.write("built %s in %.1fs\n" % (out, time.time() - t0))
    return out


def sanitizer_runtime():
    """Path of the sanitizer runtime the host-sanitized library needs preloaded."""
    out = subprocess.check_output(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
