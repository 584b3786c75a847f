"""Builds the test-only host emulation of the library (emu_hip.h): the library's sources, with the
few device-only constructs rewritten, compiled for the host with clang++ together with the fiber
runtime and four drivers (run_chains, serve_chains, ising_chains, multi_chains).

Rewrites (applied to copies under tests/emu/_build/<variant>/src, never to the sources):
  * the dynamic LDS declaration becomes the emulated workgroup's LDS buffer;
  * `s_waitcnt lgkmcnt(0)` and the empty compiler barrier that order a wavefront's LDS accesses
    become wavefront barriers;
  * the LDS and global address-space attributes are dropped.
Variants: plain (-O2), asan (AddressSanitizer), tsan (ThreadSanitizer with fiber annotations).
"""
import concurrent.futures
import glob
import hashlib
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2106_00712_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

FLAGS = {
    "plain": ["-O2", "-g"],
    "asan": ["-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-DEMU_ASAN"],
    "tsan": ["-O1", "-g", "-fsanitize=thread", "-DEMU_TSAN"],
}

DRIVERS = ("run_chains", "serve_chains", "ising_chains", "multi_chains")

REWRITES = [
    (re.compile(r"extern __shared__ double lds\[\];"), "double* lds = emu::dyn_lds();"),
    (re.compile(r'asm volatile\("s_waitcnt lgkmcnt\(0\)" ::: "memory"\);'), "emu::wave_sync();"),
    (re.compile(r'asm volatile\("" ::: "memory"\);'), "emu::wave_sync();"),
    (re.compile(r"#define DQMC_LDS __attribute__\(\(address_space\(3\)\)\)"), "#define DQMC_LDS"),
    (re.compile(r"#define DQMC_GLB __attribute__\(\(address_space\(1\)\)\)"), "#define DQMC_GLB"),
]


def compiler():
    for c in ("clang++", "/opt/rocm/llvm/bin/clang++"):
        if shutil.which(c):
            return shutil.which(c)
    return None


def _sources():
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp")) +
                   glob.glob(os.path.join(INCLUDE, "*.h")))
    return files


def _digest(variant):
    h = hashlib.sha256(variant.encode())
    for f in _sources() + sorted(glob.glob(os.path.join(HERE, "*.cpp")) + glob.glob(os.path.join(HERE, "*.h")) +
                                 [os.path.abspath(__file__)]):
        h.update(f.encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _copy_sources(dst):
    os.makedirs(dst, exist_ok=True)
    for f in _sources():
        text = open(f).read()
        for pat, rep in REWRITES:
            text = pat.sub(rep, text)
        if "asm volatile" in text or "address_space" in text:
            raise RuntimeError(f"{f}: a device-only construct has no host rewrite")
        with open(os.path.join(dst, os.path.basename(f)), "w") as out:
            out.write(text)


def build(variant="plain"):
    """Returns {driver name: executable path} for the variant, building if needed (one build at a
    time per variant, across processes)."""
    import fcntl
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    with open(os.path.join(HERE, "_build", variant + ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        return _build(variant)


def _build(variant):
    cxx = compiler()
    if cxx is None:
        raise RuntimeError("clang++ not found")
    out = os.path.join(HERE, "_build", variant)
    exes = {k: os.path.join(out, k) for k in DRIVERS}
    stamp = os.path.join(out, "stamp")
    dig = _digest(variant)
    if all(os.path.exists(p) for p in exes.values()) and os.path.exists(stamp) and open(stamp).read() == dig:
        return exes
    shutil.rmtree(out, ignore_errors=True)
    src = os.path.join(out, "src")
    _copy_sources(src)
    flags = FLAGS[variant]
    jobs = []
    for f in sorted(glob.glob(os.path.join(src, "*.hip"))):
        jobs.append([cxx, "-std=c++17", *flags, "-w", "-I", HERE, "-I", src, "-x", "c++", "-c", f,
                     "-o", f[:-4] + ".o"])
    for name in ("emu_rt",) + DRIVERS:
        jobs.append([cxx, "-std=c++17", *flags, "-w", "-I", HERE, "-I", src, "-c",
                     os.path.join(HERE, name + ".cpp"), "-o", os.path.join(out, name + ".obj")])

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(" ".join(cmd) + "\n" + r.stderr[-4000:])

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        list(ex.map(run, jobs))
    lib = sorted(glob.glob(os.path.join(src, "*.o"))) + [os.path.join(out, "emu_rt.obj")]
    # device functions defined (not inline) in the kernel headers are compiled into every
    # translation unit that includes them; the host link keeps one of the identical copies
    for name, exe in exes.items():
        run([cxx, *flags, *lib, os.path.join(out, name + ".obj"), "-o", exe, "-lpthread",
             "-Wl,--allow-multiple-definition"])
    with open(stamp, "w") as f:
        f.write(dig)
    return exes


if __name__ == "__main__":
    import sys
    print(build(sys.argv[1] if len(sys.argv) > 1 else "plain"))
