"""Build and drive the host emulation of the HIP kernels (tests/emu/).

TEST HARNESS ONLY: the kernels of paper_2006_09299_amd/csrc/ccl_pipeline.h are
compiled with g++ against tests/emu/hip_mock.h (fibers for threads and waves)
and AddressSanitizer / UBSan, so that every kernel memory access is
bounds-checked on the CPU and the results can be compared with the oracle
before any GPU run.  The product never uses this build.
"""
from __future__ import annotations

import os
import struct
import subprocess
import tempfile
from dataclasses import dataclass

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "emu", "emu.cpp")
MOCK = os.path.join(ROOT, "tests", "emu", "hip_mock.h")
PIPE = os.path.join(ROOT, "paper_2006_09299_amd", "csrc", "ccl_pipeline.h")
BUILD = os.path.join(ROOT, "tests", "emu", "_build")
EXE = os.path.join(BUILD, "ccl_emu")
# ROCm's clang: the same front end as the device compiler (and its UBSan is
# reliable with the fiber switching used by the harness)
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "clang++"

# tile configurations compiled into the emulator: (rows, columns)
TILES = {0: (32, 128), 1: (4, 64), 2: (3, 64), 3: (5, 192), 4: (64, 64), 5: (1, 64), 6: (16, 128), 7: (64, 128), 8: (32, 128),
         9: (4, 64), 10: (4, 64), 11: (4, 64), 12: (3, 64)}
# 6: 512 threads; 7: 256, relabeling 512; 8, 9: 4-adjacent foreground, 8-adjacent background;
# 10: 2 x 2 super-tiles; 11: 8 x 8 super-tiles, 4 tiles per root-reduction group; 12: 8 x 8, one tile per group


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(p) for p in (SRC, MOCK, PIPE))
    if force or not os.path.exists(EXE) or os.path.getmtime(EXE) < newest:
        os.makedirs(BUILD, exist_ok=True)
        tmp = f"{EXE}.tmp{os.getpid()}"  # parallel test workers may build at once
        subprocess.check_call([
            CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
            "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-w", "-include", MOCK, SRC, "-o", tmp,
        ])
        os.replace(tmp, EXE)
    return EXE


@dataclass
class EmuResult:
    labels: np.ndarray
    bbox: np.ndarray
    S: np.ndarray
    Sx: np.ndarray
    Sy: np.ndarray
    parent: np.ndarray
    color: np.ndarray
    n_labels: int
    euler: int


def run(images, tile_cfg: int = 0, batch: bool = False, pitch_pad: int = 0, sched: str = "fwd",
        labels: bool = True):
    """Label a list of 2-D uint8 arrays with the emulated kernels.

    sched: order in which the threads of a workgroup run after a barrier
    ("fwd", "rev", or a decimal seed for a pseudo-random order).
    labels=False: the features-only mode (no label image is written; the
    returned labels keep the fill value -7)."""
    exe = build()
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("<i", len(images)))
            for img in images:
                h, w = img.shape
                pitch = w + pitch_pad
                buf = np.zeros((h, pitch), np.uint8)
                buf[:, :w] = img
                f.write(struct.pack("<iiq", w, h, pitch))
                f.write(buf.tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", EMU_SCHED=str(sched),
                   EMU_NOLABELS="0" if labels else "1")
        p = subprocess.run([exe, str(tile_cfg), "batch" if batch else "single", fin, fout],
                           capture_output=True, text=True, env=env)
        if p.returncode != 0:
            raise RuntimeError(f"emulator failed ({p.returncode}):\n{p.stderr[-4000:]}")
        data = open(fout, "rb").read()
    out, off = [], 0
    for img in images:
        h, w = img.shape
        nl, eu = struct.unpack_from("<qq", data, off)
        off += 16
        labels = np.frombuffer(data, np.int32, h * w, off).reshape(h, w).copy()
        off += 4 * h * w
        rec = np.dtype([("f", "<i8", 7), ("pc", "<i4", 2)])
        n = max(int(nl), 0)
        tab = np.frombuffer(data, rec, n, off)
        off += rec.itemsize * n
        f = tab["f"]
        out.append(EmuResult(labels, f[:, 0:4].copy(), f[:, 4].copy(), f[:, 5].copy(), f[:, 6].copy(),
                             tab["pc"][:, 0].copy(), tab["pc"][:, 1].astype(np.uint8), int(nl), int(eu)))
    return out
