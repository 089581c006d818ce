"""Build and drive the CPU emulation of the library kernels (tests/emu/emu.cpp).

The emulator compiles the kernels' per-ray and per-node bodies for the host
(hipcc, host pass only, AddressSanitizer + UBSan on the host code) and runs them
on the same inputs the GPU path gets.  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2305_07253_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
EXE = os.path.join(BUILD, "emu")
# The same bodies with a distance-field march budget of 4 mixed iterations, so
# that nearly every ray finishes in the walk-only fall-back.
EXE_WALK = os.path.join(BUILD, "emu_walk")


def build(force: bool = False, walk: bool = False) -> str:
    exe = EXE_WALK if walk else EXE
    srcs = [os.path.join(HERE, "emu.cpp"), os.path.join(CSRC, "bvh_build.cpp")]
    deps = srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    if not force and os.path.exists(exe) and os.path.getmtime(exe) >= max(os.path.getmtime(d) for d in deps):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    tmp = exe + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           *(["-DHYB_DF_MIXED_STEPS(n)=4"] if walk else []),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stdout)
    os.replace(tmp, exe)
    return exe


def _run(hdr, par, arrays, out_bytes, walk=False):
    exe = build(walk=walk)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            np.asarray(hdr, dtype=np.int64).tofile(f)
            np.asarray(par, dtype=np.float32).tofile(f)
            for a in arrays:
                np.ascontiguousarray(a).tofile(f)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
        r = subprocess.run([exe, fin, fout], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env)
        if r.returncode != 0:
            raise RuntimeError("emulator failed (%d):\n%s" % (r.returncode, r.stdout[-4000:]))
        data = np.fromfile(fout, dtype=np.uint8)
        assert len(data) == out_bytes
        return data


def trace(verts, tris, grid, grid4, rays_soa, tmax, tau, mode=0, tmin=None, certified=False, fmt=0, tmax_ray=None,
          tau_end=0.0, walk=False):
    """Returns (t, prim, u, v, counts) exactly as the kernels compute them;
    `certified` marks the grid samples as exact distances; `fmt` stores the
    FP32 grid as F16 (1) or I8 with block scales (2), quantized by the
    oracle's definition of the formats; 3 is F16 in the kernels' two-cell
    bricks of large grids; `walk` runs the build whose march falls back to
    the cell walk after 4 iterations."""
    rays_soa = np.ascontiguousarray(rays_soa, dtype=np.float32)
    n = rays_soa.shape[1]
    N = 0 if grid is None else np.asarray(grid).shape[-1]
    g4 = np.zeros(4, np.float32) if grid4 is None else np.asarray(grid4, np.float32)
    arrays = [np.asarray(verts, np.float32), np.asarray(tris, np.int32)]
    if N:
        import oracle
        deq, stored, scales = oracle.quantize(np.asarray(grid, np.float32), 1 if fmt == 3 else fmt)
        arrays.append(deq)
        if fmt in (1, 3):
            arrays.append(stored.astype(np.float16))
        elif fmt == 2:
            arrays.append(scales.astype(np.float32))
    arrays.append(rays_soa)
    if tmin is not None:
        arrays.append(np.asarray(tmin, np.float32))
    if tmax_ray is not None:
        arrays.append(np.asarray(tmax_ray, np.float32))
    hdr = [0, n, len(verts), len(tris), N, (tmin is not None) | (2 if tmax_ray is not None else 0), mode, fmt]
    par = [tmax, tau, g4[0], g4[1], g4[2], g4[3], 1.0 if certified else 0.0, tau_end]
    raw = _run(hdr, par, arrays, 4 * n * 7, walk=walk)
    t = raw[: 4 * n].view(np.float32)
    prim = raw[4 * n: 8 * n].view(np.int32)
    u = raw[8 * n: 12 * n].view(np.float32)
    v = raw[12 * n: 16 * n].view(np.float32)
    counts = raw[16 * n:].view(np.int32).reshape(n, 3)
    return t, prim, u, v, counts


def sdf(verts, tris, grid4, N, exterior_solid=True):
    """The distance-field build kernel's node values, (N,N,N) [k,j,i]."""
    g4 = np.asarray(grid4, np.float32)
    hdr = [1, 0, len(verts), len(tris), N, 0, 0, 0]
    par = [0, 0, g4[0], g4[1], g4[2], g4[3], 1.0 if exterior_solid else 0.0, 0]
    raw = _run(hdr, par, [np.asarray(verts, np.float32), np.asarray(tris, np.int32)], 4 * N ** 3)
    return raw.view(np.float32).reshape(N, N, N)


def df_grad(grid, grid4, rays_soa, t_hit, tmax, tmin=None):
    """The backward kernel's per-ray (node[8], dt[8]) for the hits t_hit."""
    rays_soa = np.ascontiguousarray(rays_soa, dtype=np.float32)
    n = rays_soa.shape[1]
    N = np.asarray(grid).shape[-1]
    g4 = np.asarray(grid4, np.float32)
    arrays = [np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.asarray(grid, np.float32), rays_soa]
    if tmin is not None:
        arrays.append(np.asarray(tmin, np.float32))
    arrays.append(np.asarray(t_hit, np.float32))
    hdr = [2, n, 0, 0, N, 1 if tmin is not None else 0, 2, 0]
    par = [tmax, 0, g4[0], g4[1], g4[2], g4[3], 0, 0]
    raw = _run(hdr, par, arrays, 64 * n + 32 * n)
    return raw[:64 * n].view(np.int64).reshape(n, 8), raw[64 * n:].view(np.float32).reshape(n, 8)


def block_order(nb: int, run: int):
    """The kernels' workgroup-to-block map (xcd_block) for a launch of nb blocks."""
    raw = _run([3, nb, 0, 0, run, 0, 0, 0], [0] * 8, [], 4 * nb)
    return raw.view(np.uint32)
