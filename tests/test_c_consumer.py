"""The C ABI from plain C.

include/wkern.h compiles as strict C99 and C11 (and as C++11), with every
entry point it declares taken by address.  tests/c_consumer/wkern_c_consumer.c
is a C99 program that uses only that header, the HIP runtime's C API and
libwkern.so: no C++, no Python and no torch in its process.  It builds with
gcc -pedantic -Werror.  On the CPU it checks the device-independent error
path and then fails cleanly at wkern_plan, since there is no device.  On the
GPU (-m gpu) the cache and radial lines it writes are compared with the FP64
oracle at the parity gates (FP32 contraction 1e-5, split-BF16 1e-6; error =
max |K - K_ref| / max |K_ref| per plane).  The program itself checks that a
replay of the captured graph writes the same bytes as the first call.
"""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import hankel as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(ROOT, "paper_1904_08463_amd")
SRC = os.path.join(ROOT, "tests", "c_consumer", "wkern_c_consumer.c")
ROCM = "/opt/rocm"

GATE = {"fp32": 1e-5, "bf16x6": 1e-6}

needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None or
                               not os.path.isdir(os.path.join(ROCM, "include")),
                               reason="needs gcc, g++ and the ROCm headers")
needs_lib = pytest.mark.skipif(not os.path.exists(os.path.join(LIBDIR, "libwkern.so")),
                               reason="libwkern.so not built")


def _declared_functions():
    with open(os.path.join(INCLUDE, "wkern.h")) as f:
        hdr = f.read()
    return sorted(set(re.findall(r"^\S[^\n(]*?\b(wkern_[a-z_0-9]+)\s*\(", hdr, flags=re.M)))


def _build(tmp_path, std="c99"):
    exe = str(tmp_path / f"wkern_c_consumer_{std}")
    cmd = ["gcc", f"-std={std}", "-O2", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-D__HIP_PLATFORM_AMD__", "-isystem", os.path.join(ROCM, "include"), f"-I{INCLUDE}",
           SRC, f"-L{LIBDIR}", "-lwkern", f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _write_problem(path, wl, precision, mirror=None):
    hdr = np.array([wl.image_size, wl.n_radial, wl.oversampling, wl.radial_refine, wl.n_planes,
                    wl.max_support, {"fp32": 0, "bf16x6": 1}[precision],
                    {"linear": 0, "cubic": 1}[wl.interp], 0 if mirror is None else 1],
                   dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes())
        f.write(np.float64(wl.cellsize).tobytes())
        f.write(np.ascontiguousarray(wl.support, dtype=np.int32).tobytes())
        if mirror is not None:
            f.write(np.ascontiguousarray(mirror, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(wl.taper, dtype=np.float32).tobytes())
        f.write(np.ascontiguousarray(wl.w, dtype=np.float64).tobytes())


def _read_result(path, n_planes):
    raw = open(path, "rb").read()
    pos = 0
    offsets = np.frombuffer(raw, np.int64, n_planes + 1, pos).copy()
    pos += 8 * (n_planes + 1)
    nrho = np.frombuffer(raw, np.int32, n_planes, pos).copy()
    pos += 4 * n_planes
    cache = np.frombuffer(raw, np.complex64, int(offsets[-1]), pos).copy()
    pos += 8 * int(offsets[-1])
    lines = np.frombuffer(raw, np.complex128, int(nrho.sum()), pos).copy()
    pos += 16 * int(nrho.sum())
    assert pos == len(raw), "result file size"
    return offsets, nrho, cache, lines


def _mirrored_workload():
    """Ragged random planes plus three planes at -w of the first three
    (declared as mirrors: written as conjugates, their w not read)."""
    wl = W.random_small(11, n_planes=10, n_radial=160, os_=4, max_support=25)
    k = 3
    wl.w = np.concatenate([wl.w, -wl.w[:k]])
    wl.support = np.concatenate([wl.support, wl.support[:k]]).astype(np.int32)
    mirror = np.concatenate([np.full(10, -1), np.arange(k)]).astype(np.int32)
    return wl, mirror


@needs_gcc
@pytest.mark.parametrize("std", ["c99", "c11"])
def test_header_compiles_as_strict_c(tmp_path, std):
    funcs = _declared_functions()
    assert len(funcs) > 20
    src = tmp_path / "every_entry_point.c"
    src.write_text('#include "wkern.h"\n'
                   "typedef void (*any_fn)(void);\n"
                   "int main(void) {\n"
                   "  volatile any_fn fns[] = {\n" +
                   "".join(f"    (any_fn){f},\n" for f in funcs) +
                   "  };\n"
                   "  return (int)(sizeof(fns) / sizeof(fns[0])) > 0 ? 0 : 1;\n"
                   "}\n")
    r = subprocess.run(["gcc", f"-std={std}", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-Wno-cast-function-type", f"-I{INCLUDE}", "-fsyntax-only", str(src)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]


@needs_gcc
def test_header_compiles_as_cpp(tmp_path):
    funcs = _declared_functions()
    src = tmp_path / "every_entry_point.cpp"
    src.write_text('#include "wkern.h"\n'
                   "using any_fn = void (*)();\n"
                   "int main() {\n"
                   "  volatile any_fn fns[] = {\n" +
                   "".join(f"    reinterpret_cast<any_fn>(&{f}),\n" for f in funcs) +
                   "  };\n"
                   "  return wkern_abi_version() == WKERN_ABI_VERSION && fns[0] ? 0 : 1;\n"
                   "}\n")
    r = subprocess.run(["g++", "-std=c++11", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        f"-I{INCLUDE}", "-fsyntax-only", str(src)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]


@needs_gcc
@needs_lib
def test_c_consumer_fails_cleanly_without_a_device(tmp_path):
    exe = _build(tmp_path)
    wl = W.precision()
    prob, res = str(tmp_path / "problem.bin"), str(tmp_path / "result.bin")
    _write_problem(prob, wl, "bf16x6")
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="", WKERN_FAULT="")
    r = subprocess.run([exe, prob, res], capture_output=True, text=True, timeout=120, env=env)
    # the invalid-description and layout checks come first and need no device
    assert r.returncode == 1, (r.stdout + r.stderr)[-4000:]
    assert "wkern_plan:" in r.stderr, r.stderr[-4000:]
    assert "invalid description" not in r.stderr and "disagree" not in r.stderr
    assert not os.path.exists(res)


@pytest.mark.gpu
@needs_gcc
@needs_lib
@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_c_consumer_matches_oracle(tmp_path, precision):
    exe = _build(tmp_path)
    wl, mirror = _mirrored_workload()
    P = wl.n_planes
    prob, res = str(tmp_path / "problem.bin"), str(tmp_path / "result.bin")
    _write_problem(prob, wl, precision, mirror)
    print(f"case c-consumer precision={precision} P={P} Nr={wl.n_radial}", flush=True)
    r = subprocess.run([exe, prob, res], capture_output=True, text=True, timeout=120)
    print(r.stdout.strip(), flush=True)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    offsets, nrho, cache, lines = _read_result(res, P)

    ref_offsets = np.zeros(P + 1, dtype=np.int64)
    ref_offsets[1:] = np.cumsum(wl.oversampling ** 2 * wl.support.astype(np.int64) ** 2)
    assert np.array_equal(offsets, ref_offsets)
    caches, ref_lines = H.generate_workload(wl)
    loffs = np.concatenate([[0], np.cumsum(nrho)])
    worst_c = worst_l = 0.0
    for p in range(P):
        assert nrho[p] == len(ref_lines[p])
        got = cache[offsets[p]:offsets[p + 1]].reshape(caches[p].shape)
        ec = float(np.max(np.abs(got - caches[p])) / np.max(np.abs(caches[p])))
        el = float(np.max(np.abs(lines[loffs[p]:loffs[p + 1]] - ref_lines[p])) /
                   np.max(np.abs(ref_lines[p])))
        worst_c, worst_l = max(worst_c, ec), max(worst_l, el)
        assert ec <= GATE[precision], f"plane {p}: cache error {ec:.3e}"
        assert el <= GATE[precision], f"plane {p}: radial error {el:.3e}"
    # a mirrored plane and its line are the exact conjugates of its source's
    for p in range(P):
        if mirror[p] >= 0:
            q = int(mirror[p])
            assert np.array_equal(cache[offsets[p]:offsets[p + 1]],
                                  np.conj(cache[offsets[q]:offsets[q + 1]]))
            assert np.array_equal(lines[loffs[p]:loffs[p + 1]],
                                  np.conj(lines[loffs[q]:loffs[q + 1]]))
    print(f"c-consumer/{precision}: worst cache error {worst_c:.3e}, radial {worst_l:.3e}",
          flush=True)
