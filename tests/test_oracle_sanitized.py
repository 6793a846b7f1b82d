"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) renders small versions of every workload family without a
report: pinhole box room, confocal scan with cosine and NLOS area sampling
(including deeper paths), fog with GGX spheres, the glass room with
scattering delays, the phasor film, the forward-mode derivative and the
adjoint.  The renders run in a child process that preloads the ASan
runtime (ASan must come first in the process); UBSan aborts on the first
finding (-fno-sanitize-recover)."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    from paper_2510_25660_amd import scenes
    with oracle.using_library(LIB):
        sc = scenes.box_scene(width=8, height=8)
        O = oracle.Oracle(sc)
        O.render(spp=4, threads=2)
        O.render_phasor([0.5, 3.0], spp=2)
        O.render_tangent(np.ones(sc.n_tris), None, spp=2)
        nl = scenes.confocal_nlos(grid=4, n_tris=500, spp=64)
        On = oracle.Oracle(nl)
        On.render(threads=2)
        On.render(nlos_area=True)
        On.render(nlos_area=True, max_depth=5, spp=16)
        fog = scenes.large_scene(cells=8, sphere_freq=3, grid=2, width=8, height=6, n_bins=64, bin_width=0.05, spp=2)
        Of = oracle.Oracle(fog)
        Of.render()
        Of.records(np.arange(8))
        gl = scenes.glass_box_scene(delay_mean=0.05, width=8, height=8, spp=4)
        oracle.Oracle(gl).render()
        d = scenes.diff_scene(sub=2, width=8, height=8, spp=4)
        Od = oracle.Oracle(d)
        film, _, _ = Od.render(frozen=True)
        Od.backward(np.ascontiguousarray(film, np.float32).reshape(d.n_pixels, d.n_bins), frozen=True,
                    want_primal=True)
    print("SANITIZED_OK")
""")


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(oracle_mod, tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    so = str(tmp_path / "liboracle_san.so")
    flags = [f for f in oracle_mod.CFLAGS if f != "-O2"] + ["-O1", "-g", "-fno-omit-frame-pointer",
                                                             "-fsanitize=address,undefined",
                                                             "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, "-o", so, oracle_mod.SRC_PATH, "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + ((":" + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    code = SCRIPT.replace("ROOT", repr(ROOT)).replace("LIB", repr(so))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
