"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host C/C++ code (no GPU).

The C oracle (oracle/uhm_oracle.c: Algorithms 5 and 6) and the host builder
(csrc/builder_native.cpp: dense blocks, ACA with partial pivoting, the direct
construction's per-block ACA, the scaled copies that lay out the H factors) are compiled with -fsanitize=address,undefined and no error
recovery, and a child Python process loads those builds (the ASan runtime preloaded) and
runs them on small ragged clouds: the two-phase and direct builders, and Algorithms 5 and 6
at 1 and 3 threads, checked against the block-wise definitions.  Any invalid access or
undefined behaviour aborts the child, and the test fails with its report.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, {root!r})
    from oracle import uniform
    from paper_2405_15573_amd import builder, inputs
    for surface, n, leaf, seed in (("sphere", 700, 32, 1), ("cube", 650, 32, 2), ("ellipsoid", 900, 32, 3)):
        cloud = inputs.make_cloud(surface, n, seed=seed)
        op = builder.build_operator(cloud, leaf=leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
        od = builder.build_uniform_direct(cloud, leaf=leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
        x = inputs.make_rhs(cloud.n, 2, seed=seed)
        y = uniform.uh_mvp(vars(op), x)
        for th in (1, 3):
            y6 = uniform.alg6(vars(op), x, nthreads=th)
            y5 = uniform.alg5(vars(op), x, nthreads=th)
            assert np.linalg.norm(y6 - y) <= 1e-13 * np.linalg.norm(y), (surface, th)
            assert np.linalg.norm(y5 - uniform.h_mvp(vars(op), x)) <= 1e-13 * np.linalg.norm(y), (surface, th)
        yd = uniform.uh_mvp(vars(od), x)
        assert np.linalg.norm(yd - y) <= 1e-10 * np.linalg.norm(y), surface
        print("ok", surface, cloud.n, flush=True)
    print("loaded", builder._native()._name, uniform._lib()._name, flush=True)
""")


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_host_code_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the gcc AddressSanitizer runtime is not installed")
    oracle_so = str(tmp_path / "liboracle_san.so")
    builder_so = str(tmp_path / "libuhm_builder_san.so")
    _compile(["gcc", "-std=c99", "-fopenmp", "-fPIC", "-shared", *SAN, os.path.join(ROOT, "oracle", "uhm_oracle.c"),
              "-o", oracle_so])
    _compile(["g++", "-std=c++17", "-fopenmp", "-fPIC", "-shared", *SAN,
              os.path.join(ROOT, "paper_2405_15573_amd", "csrc", "builder_native.cpp"), "-o", builder_so])
    env = dict(os.environ, LD_PRELOAD=asan, UHM_ORACLE_LIB=oracle_so, UHM_BUILDER_LIB=builder_so,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="3")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=900)
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, report
    assert r.stdout.count("ok ") == 3, report
    assert f"loaded {builder_so} {oracle_so}" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
