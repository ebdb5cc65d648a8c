"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
a driver runs every oracle function on the tiny workload's scene and rays; the run must end
cleanly (no out-of-bounds access, leak or undefined operation) and agree with the regular
build's results."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "hcc_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *SRC, "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    spec = W.tiny_scene()
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, 32, 32)
    ph = O.trace(ob, prim)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=2, bounce=0)
    rays = np.ascontiguousarray(np.concatenate([sec, prim]), np.float32)
    # a camera ray straight down: 1/0 = inf on two axes in every slab test (its origin lies on no box plane)
    rays[sec.shape[0] + 5, 4:7] = [0.0, 0.0, -1.0]
    (tmp_path / "tris.bin").write_bytes(np.ascontiguousarray(spec.tris, np.float32).tobytes())
    (tmp_path / "rays.bin").write_bytes(rays.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe), str(tmp_path / "tris.bin"), str(tmp_path / "rays.bin")], capture_output=True,
                       text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    n, m, agree, occ_agree, _, anc, f0, f1, morton = r.stdout.split()
    assert int(n) == spec.tris.shape[0] and int(m) == rays.shape[0]
    # the sanitized build computes what the regular one does
    assert int(agree) == int(occ_agree) == rays.shape[0]
    cb = O.cut_boxes(ob, O.select_cut(ob, O.had(ob), 64))
    keys = O.encode_hcc(rays, cb, 32)
    perm = O.sort(keys)
    assert abs(float(anc) - O.anc(keys, perm, 32)) < 1e-6
    for order, f in ((0, f0), (1, f1)):
        wn, wt, _ = O.wave_fetches(ob, rays, perm, 64, True, order)
        assert int(f) == int(wn.sum() + wt.sum())
    assert int(morton) == O.morton3(1, 2, 3)
