"""Address and undefined-behaviour sanitizer builds of the host code, on the
CPU: the FP64 oracle (oracle/*.c) and the C-ABI host side of the GPU library
(api.cpp, tsdf_api.cpp, with host-only stand-ins for the device symbols in
tests/c/device_stubs.cpp) are compiled with gcc/g++ -fsanitize=address,undefined
and exercised in a child process (the sanitizer runtime preloaded); any
report fails the test.  Without a GPU the library's calls end at their
argument checks or at the first HIP call, which is where its host logic
lives."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _libasan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc has no AddressSanitizer runtime")
    return path


def _run(tmp_path, script):
    env = dict(os.environ, LD_PRELOAD=_libasan(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], capture_output=True, text=True, env=env,
                       cwd=str(tmp_path), timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "Sanitizer" not in out and "runtime error" not in out, out[-6000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("psweep_oracle.c", "tsdf_oracle.c")]
    subprocess.check_call(["gcc", *SAN, "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           *srcs, "-o", str(lib), "-lm"])
    out = _run(tmp_path, f"""
        import numpy as np
        import oracle
        oracle._LIB_PATH = {str(lib)!r}
        import scenegen
        from scenegen import Level, Settings
        fr = scenegen.random_small_frame(w=40, h=32, n_src=2, seed=3, f=26.0)
        lv = Level(n_fronto=6, near=1.0, far=20.0, n_ground=4, h_lo=-0.3, h_hi=0.3, window=5)
        st = Settings(levels=[lv], best_k=2)
        r = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, volume=True,
                               srcvol=True, srcsig=True)
        assert (r["index"] >= 0).sum() > 50
        st2 = Settings(levels=[Level(n_fronto=6, near=1.0, far=20.0, window=5, downsample=2),
                               Level(n_fronto=4, near=5.0, far=30.0, window=5, crop=(8, 8, 20, 16))], best_k=2)
        m = oracle.run(fr, st2)["merged"]
        soft = Settings(levels=[Level(n_fronto=6, near=1.0, far=20.0, window=5)], best_k=2, mode="soft",
                        temperature=0.1)
        rho, lse = oracle.soft_forward(soft.levels[0], soft, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses)
        g = np.random.default_rng(0).normal(size=(8, 10))
        gs, gp = oracle.soft_backward(soft.levels[0], soft, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses,
                                      (12, 10, 10, 8), g)
        print("soft argmin", oracle.soft_argmin([0.3, float("nan"), 0.2], [0.1, 0.2, 0.3], 0.1))
        d, c = oracle.depth_filter(fr.ref_cam, st.ground_n, r["depth"], r["cost1"], r["cost2"])
        oracle.mask_boxes(d, [(2, 2, 9, 9), (30, 20, 60, 40)], code=c)
        seq = scenegen.depth_sequence(n_frames=2, w=40, h=32, step_m=0.5, seed=4)
        o = oracle.TsdfOracle(0.1, 0.3, (6, 4, 8), min_obs=1)
        for P, cen, dm in zip(seq.poses, seq.centres, seq.depths):
            o.integrate(seq.cam, P, dm, (cen[0], cen[1], cen[2] + 2.0))
        print("tsdf voxels", int(np.isfinite(o.extract()).sum()))
        print("oracle ok")
    """)
    assert "oracle ok" in out


def test_abi_host_code_under_sanitizers(tmp_path):
    if subprocess.run(["bash", "-c", "ls /opt/rocm/lib/libamdhip64.so"], capture_output=True).returncode:
        pytest.skip("no HIP runtime library")
    csrc = os.path.join(ROOT, "paper_1809_06132_amd", "csrc")
    lib = tmp_path / "libpsweep_host_san.so"
    cmd = ["g++", "-std=c++17", "-fPIC", "-shared", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(csrc, "api.cpp"), os.path.join(csrc, "tsdf_api.cpp"),
           os.path.join(ROOT, "tests", "c", "device_stubs.cpp"), "-o", str(lib),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.check_call(cmd)
    out = _run(tmp_path, f"""
        import ctypes
        from paper_1809_06132_amd import psweep
        psweep.LIB_PATH = {str(lib)!r}
        L = psweep.lib()
        import tests.test_abi as t
        # every rejected configuration of the CPU ABI tests, then a valid one
        # (it gets as far as the pinned staging allocation, which needs a GPU)
        bad = list(t.test_create_rejects_bad_config.pytestmark[0].args[1])
        for kw, status in bad:
            try:
                psweep.psweep_create(t._cfg(psweep, **kw))
                raise SystemExit("accepted " + repr(kw))
            except psweep.PsweepError as e:
                assert e.status == status, (kw, e.status)
        try:
            psweep.psweep_create(t._cfg(psweep))
        except psweep.PsweepError as e:
            assert e.status in (psweep.EHIP,), e.status
        assert L.psweep_create(None, None) == psweep.EINVAL
        assert L.psweep_run(None, None, 0, None, None) == psweep.EINVAL
        assert L.psweep_run_noalloc(None, None, 0, None, None) == psweep.EINVAL
        assert L.psweep_soft_depth_backward(None, None, None, None, None) == psweep.EINVAL
        assert L.psweep_mask_boxes(None, 0, None, None, 0, 0, None, None) == psweep.EINVAL
        assert L.psweep_plane_pixels_met(None, None, 0, None) == psweep.EINVAL
        print(psweep.psweep_version(), psweep.psweep_last_error(None))
        c = psweep.psweep_tsdf_config(0.1, 0.3, (psweep._i32 * 3)(8, 4, 8), 100.0, 3, 320, 256)
        try:
            psweep.psweep_tsdf_create(c)
        except psweep.PsweepError as e:
            print("tsdf create without a GPU:", e.status)
        print("host ok")
    """)
    assert "host ok" in out
