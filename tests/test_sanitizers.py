"""AddressSanitizer + UndefinedBehaviorSanitizer builds, exercised on the CPU.

* The oracle (``oracle/oracle.cpp``), built with g++ ``-O1 -fsanitize=address,
  undefined``, runs every entry point on small scenes (pinhole and
  orthographic, SH degrees 0 and 3) in a child process with the sanitizer
  runtime preloaded.
* The library (every ``csrc/*.hip`` source, the sanitizers on the host side
  only) is loaded the same way and its
  GPU-free entry points are called: camera layout, workspace sizes, option
  checks, status strings and the argument checks of every stage.

Any sanitizer report, or a non-zero exit, fails the test.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _run_child(code, preload, extra_env):
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2", **extra_env)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return r.stdout


ORACLE_SCRIPT = r"""
import numpy as np
from paper_2505_05587_amd import scenes
from tests.helpers import tiny_scene
from oracle import oracle as O
for model, deg in ((0, 0), (1, 0), (0, 3)):
    P, cams, target = tiny_scene(7 + model + deg, 30, 24, sh_degree=deg, model=model)
    opts = scenes.opts("3dgs", bg=(0.1, 0.2, 0.3))
    pr = O.project(P, deg, cams, opts)
    keys, vals, ranges = O.sort(P, deg, cams, opts)
    ref = O.forward_backward(P, deg, cams, opts, target)
    O.forward_backward(P, deg, cams, opts, target, per_view=True)
    O.forward_backward(P, deg, cams, opts, dl_dimage=np.ones(3 * cams.total_pixels()))
    O.loss(P, deg, cams, opts, target)
    pix = np.arange(0, cams.total_pixels(), 7)
    O.render_pixels(P, deg, cams, opts, pix)
    O.grads_sampled(P, deg, cams, opts, target, np.arange(0, P.shape[1], 3), flagged=True)
    npx = len(pix)
    O.pixel_variants(P, deg, cams, opts, target, pix, -np.ones(npx, np.int32), np.full((npx, 3), 2))
    O.tile_lists(P, deg, cams, opts, np.arange(min(4, len(ranges))))
    d = O.densify(P, deg, ref["S"], 1.0, 0.01, -1e-6, budget=3)
    O.split_remap(np.ones_like(P, dtype=np.float64), d["split"])
    O.adam_step(P.astype(np.float64), ref["grads"], np.zeros(P.shape), np.zeros(P.shape), 1, [1e-3] * 6)
    if deg == 0:
        S21 = O.split6(P, deg, cams, opts, target)
        O.densify6(P, deg, S21, 1.0, 0.01, -1e-6)
    O.loss_merged_split(P, deg, cams, opts, target, 0, np.array([1e-3, 0.0, 0.0]), 0.01)
O.sh_basis(3, np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]]))
print("oracle ok")
"""


@pytest.mark.timeout(900)
def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(ROOT, "oracle", "oracle.cpp")])
    out = _run_child(ORACLE_SCRIPT, f"{asan}:{ubsan}", {"STEEPGS_ORACLE_LIB": lib})
    assert "oracle ok" in out


ABI_SCRIPT = r"""
import ctypes as C
import numpy as np
from paper_2505_05587_amd import _lib as L, scenes
lib = L.lib()
# camera layout and workspace sizes for a few tile shapes and view counts
for tw, th in ((16, 16), (16, 8), (8, 8)):
    for V in (1, 3, 16):
        cams = scenes.make_cameras([(0.0, 0.0, 3.0 + k) for k in range(V)], [(97 + 13 * k, 61 + 7 * k) for k in range(V)])
        o = L.make_opts(dict(scenes.opts("3dgs"), tile_w=tw, tile_h=th))
        arr = (L.Camera * V)()
        for v in range(V):
            arr[v].fx, arr[v].fy, arr[v].cx, arr[v].cy = float(cams.fx[v]), float(cams.fy[v]), float(cams.cx[v]), float(cams.cy[v])
            arr[v].width, arr[v].height, arr[v].model = int(cams.width[v]), int(cams.height[v]), int(cams.model[v])
        px, tt = L.steepgs_layout_cameras(arr, o)
        assert px == int(sum(int(w) * int(h) for w, h in zip(cams.width, cams.height)))
        assert tt == int(sum(-(-int(w) // tw) * -(-int(h) // th) for w, h in zip(cams.width, cams.height)))
        for stage in range(0, 7):
            lib.steepgs_workspace_size(stage, 1000, V, 1 << 20, tt)
# argument checks of every stage (no device memory touched)
o = L.make_opts(scenes.opts("3dgs"))
bad = L.make_opts(dict(scenes.opts("3dgs"), tile_w=12))
assert lib.steepgs_project(None, -1, 0, None, 1, C.byref(o), None, None, None, None) == L.ERR_INVALID_ARG
assert lib.steepgs_project(None, 10, 0, None, 1, C.byref(bad), None, None, None, None) == L.ERR_INVALID_ARG
for code in range(-2, 12):
    s = lib.steepgs_status_string(code)
print("abi ok")
"""


@pytest.mark.timeout(900)
def test_host_abi_under_asan_ubsan(tmp_path):
    asan = _clang_asan()
    if not asan or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang ASan runtime not installed")
    # device code as in the product build, the sanitizers on the host side only
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2505_05587_amd", "csrc", "*.hip")))
    objs = [str(tmp_path / (os.path.basename(src) + ".o")) for src in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda so: subprocess.check_call([HIPCC, *flags, "-c", so[0], "-o", so[1]],
                                                     stderr=subprocess.DEVNULL), zip(srcs, objs)))
    lib = str(tmp_path / "libsteepgs_san.so")
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libasan",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs,
                           "-o", lib])
    out = _run_child(ABI_SCRIPT, asan, {"STEEPGS_LIB": lib})
    assert "abi ok" in out
