"""Host build of the batched solver's kernel (k_batched.hip) for tests.

build() compiles the library's kernel source and host plan as host C++ with
the emulation header under AddressSanitizer (clang); run_batched() writes a
batch to a file, runs the build in a subprocess with a time limit and reads
the outputs back. Test infrastructure only: the library never uses it."""
import os
import shutil
import struct
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2312_09376_amd", "csrc")
OUT_DIR = os.path.join(ROOT, "_build", "hostemu")
EXE = os.path.join(OUT_DIR, "emu_batched")


def clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def _inputs(kernel_src, csrc):
    return [kernel_src, os.path.join(csrc, "batch_plan.cpp"), os.path.join(csrc, "internal.h"),
            os.path.join(csrc, "butterfly_dev.h"), os.path.join(csrc, "mma16.h"),
            os.path.join(ROOT, "include", "rbt.h"), os.path.join(HERE, "emu_runtime.cpp"),
            os.path.join(HERE, "emu_batched.cpp"), os.path.join(HERE, "include", "hip", "hip_runtime.h"),
            os.path.abspath(__file__)]


def build(kernel_src=None, exe=EXE, csrc=CSRC, force=False):
    """Compile (kernel_src defaults to the library's k_batched.hip) unless
    the executable is newer than every input. Returns its path."""
    cc = clang()
    if cc is None:
        raise RuntimeError("clang++ not found")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    kernel_src = kernel_src or os.path.join(csrc, "k_batched.hip")
    if not force and os.path.exists(exe):
        t = os.path.getmtime(exe)
        if all(os.path.getmtime(f) < t for f in _inputs(kernel_src, csrc) if os.path.exists(f)):
            return exe
    cmd = [cc, "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-Wno-psabi", f"-I{os.path.join(HERE, 'include')}", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{csrc}", "-x", "c++", kernel_src, os.path.join(csrc, "batch_plan.cpp"),
           os.path.join(HERE, "emu_runtime.cpp"), os.path.join(HERE, "emu_batched.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError("host build failed:\n" + r.stderr[-4000:])
    return exe


def run_batched(As, Bs, depth=2, prec=0, seed=1, tol=-10.0, max_iter=10, ct2_min_n=2 ** 63 - 1,
                grid=None, granule=1, kind=0, sides=2, exe=EXE, timeout=300, workdir=None,
                threads=8):
    """Solve the batch with the host build. Returns (Xs, iters, berr, info,
    path, checks) with checks = {"divergent_barriers", "ticket", "plan_intact"}
    (ticket: the queue word after the launch); raises RuntimeError with the build's report
    (sanitizer or emulator) if it fails, subprocess.TimeoutExpired if it
    does not finish."""
    batch = len(As)
    ns = np.array([a.shape[0] for a in As], dtype=np.int64)
    ks = np.array([b.shape[1] for b in Bs], dtype=np.int64)
    grid = grid or max(1, min(batch, 512))
    workdir = workdir or OUT_DIR
    os.makedirs(workdir, exist_ok=True)
    fin = os.path.join(workdir, f"in_{os.getpid()}.bin")
    fout = os.path.join(workdir, f"out_{os.getpid()}.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<9q", batch, depth, prec, max_iter, ct2_min_n, grid, granule, kind, sides))
        f.write(struct.pack("<Qd", seed, tol))
        f.write(ns.tobytes())
        f.write(ks.tobytes())
        for a, b in zip(As, Bs):
            f.write(np.asfortranarray(a, dtype=np.float64).tobytes(order="F"))
            f.write(np.asfortranarray(b, dtype=np.float64).tobytes(order="F"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               EMU_THREADS=str(threads))
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout, env=env)
    os.remove(fin)
    if r.returncode:
        raise RuntimeError(f"host build exited with {r.returncode}:\n{r.stderr[-6000:]}")
    raw = open(fout, "rb").read()
    os.remove(fout)
    off = 0
    Xs = []
    for n, k in zip(ns, ks):
        cnt = int(n * k)
        Xs.append(np.frombuffer(raw, np.float64, cnt, off).reshape((int(k), int(n))).T.copy())
        off += 8 * cnt
    iters = np.frombuffer(raw, np.int32, batch, off); off += 4 * batch
    berr = np.frombuffer(raw, np.float64, batch, off); off += 8 * batch
    info = np.frombuffer(raw, np.int32, batch, off); off += 4 * batch
    path = np.frombuffer(raw, np.int32, batch, off); off += 4 * batch
    div, ticket, intact = struct.unpack_from("<QqQ", raw, off)
    checks = {"divergent_barriers": div, "ticket": ticket, "plan_intact": bool(intact)}
    return Xs, iters.copy(), berr.copy(), info.copy(), path.copy(), checks
