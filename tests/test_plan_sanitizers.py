"""The threaded float64 host plan builder under the host sanitizers: built with
AddressSanitizer + UndefinedBehaviorSanitizer and, separately, ThreadSanitizer (host code
only, the ROCm clang), it plans a set of geometries -- the parity case with and without
helix offsets, the half-sample grid, a non-commensurate grid, a ragged grid and the
sparse-detector workload -- on 8 worker threads; every run must end cleanly with no
sanitizer report, and print the counts the library's own build reports."""
import os
import subprocess

import pytest

from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/lib/llvm/bin/clang++"
SRC = [os.path.join(ROOT, "paper_2201_02309_amd", "csrc", "plan.cpp"),
       os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"),
       os.path.join(ROOT, "tests", "sanitize", "device_stubs.cpp")]


def _line(wl, grid=None, flags=0, kz=0):
    g = wl.geom.as_dict()
    gr = grid or wl.grid.as_dict()
    vals = [g["R"], g["D"], g["feed_per_turn"], g["lambda0"], g["z0"], g["lambda_first"],
            g["dalpha"], g["col_offset"], g["dw"], g["row_offset"], g["n_views"],
            g["views_per_turn"], g["det_cols"], g["det_rows"], gr["dx"], gr["dy"], gr["dz"],
            gr["x_first"], gr["y_first"], gr["z_first"], gr["nx"], gr["ny"], gr["nz"],
            0, 8, flags, kz]
    return " ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in vals)


def _cases():
    return [(configs.config1(), {}),
            (configs.with_helix_offsets(configs.config1()), {}),
            (configs.config1(), {"flags": 1, "kz": 8}),
            (configs.tiny(nxy=20, nz=9, slices_per_pitch=None, feed=23.0, dxy=2.1), {"kz": 32}),
            (configs.tiny(nxy=13, nz=29, cols=48, rows=8, views_per_turn=72, turns=3, feed=24.0,
                          dxy=2.0, slices_per_pitch=12), {}),
            (configs.config3(0), {})]


def _build(tmp, name, flags):
    if not os.path.exists(CXX) or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("ROCm clang++ / HIP runtime not available")
    exe = os.path.join(tmp, name)
    cmd = [CXX, "-x", "c++", "-O1", "-g", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-fno-omit-frame-pointer"] + flags + SRC + [
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr + r.stdout).lower():
        pytest.skip("sanitizer runtime unavailable: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.parametrize("kind", ["address+undefined", "thread"])
def test_host_plan_builder_under_sanitizers(tmp_path, kind):
    flags = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
             if kind == "address+undefined" else ["-fsanitize=thread"])
    exe = _build(str(tmp_path), "plan_" + kind.split("+")[0], flags)
    cases = _cases()
    stdin = "\n".join(_line(wl, **kw) for wl, kw in cases) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input=stdin, capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert r.returncode == 0, out[-4000:]
    for bad in ("AddressSanitizer", "runtime error", "ThreadSanitizer", "LeakSanitizer"):
        assert bad not in out, out[-4000:]
    assert f"plans {len(cases)} ok" in r.stdout
    # the counts agree with the library's own (uninstrumented) build of the same plans
    import paper_2201_02309_amd as K
    lines = [l for l in r.stdout.splitlines() if l.startswith("plan ")]
    for (wl, kw), l in zip(cases, lines):
        p = K.Plan(wl.geom.as_dict(), wl.grid.as_dict(), bind=False, half_sample=kw.get("flags") == 1,
                   bp_slices=kw.get("kz", 0))
        assert f"n_vv {p.info['n_vv']} " in l and f"valid {p.info['n_valid_voxels']} " in l, l
        p.close()
