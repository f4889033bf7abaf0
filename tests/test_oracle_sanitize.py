"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc), driven through its Python front end in a child process over every
entry point: steps in the three likelihood modes, RNA and ARNA, the
information-sharing start, tracing with ambiguous centres, the ring (plain
and grouped), N_ex, resampling, the gradient and its replay (Gaussian patch
likelihood).  Any invalid
access or undefined operation aborts the child."""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "arna_oracle.c")

DRIVER = textwrap.dedent("""
    import numpy as np
    from oracle import oracle as orc
    from paper_1310_4624_amd import synth
    rng = np.random.Generator(np.random.PCG64(3))
    base = dict(patch=9, init_mode=0, fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99,
                psf_sigma=1.5, background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5, seed=9)
    cases = [
        dict(base, n_filters=2, n_pe=4, n_per_pe=100, width=48, height=40, mode=1, lik_mode=0),
        dict(base, n_filters=1, n_pe=5, n_per_pe=77, width=40, height=40, mode=0, lik_mode=0,
             init_mode=1),
        dict(base, n_filters=1, n_pe=3, n_per_pe=64, width=32, height=32, mode=1, lik_mode=2,
             background=10.0),
        dict(base, n_filters=2, n_pe=4, n_per_pe=50, width=64, height=64, mode=1, lik_mode=1,
             noise_sigma=1.0),
        dict(base, n_filters=1, n_pe=6, n_per_pe=40, width=32, height=32, mode=1, lik_mode=0,
             patch=7),
    ]
    for cfg in cases:
        F, W, H = cfg["n_filters"], cfg["width"], cfg["height"]
        if cfg["lik_mode"] == 1:
            truth, frames = synth.point_sequence(5, F, 4)
            truth = truth[0]
        else:
            truth = np.zeros((F, 5), np.float32)
            truth[:, 0], truth[:, 1], truth[:, 4] = 4.0, H - 5.0, 10.0   # near a corner
            truth[:, 2] = 0.3
            frames = np.stack([synth.render(truth.astype(np.float64), W, H, 1.5,
                                            cfg["background"], 2.0, rng) for _ in range(4)])
        o = orc.Oracle(cfg, truth)
        o.set_ambiguity(4 * 2.0 ** -23, 2e-5)
        for k in range(4):
            tr = o.step(frames[k])
            assert tr["status"] == 0, tr["status"]
        s, L, k = o.get_state()
        o.set_state(s, L, k)
        o.step(frames[0], trace=False)
        if cfg["lik_mode"] == 0:   # the gradient covers the Gaussian patch likelihood
            J, dJ, tape = orc.grad(cfg, truth, frames[:3])
            orc.replay(cfg, truth, frames[:3], tape, dI0=0.01)
        M, n_p = cfg["n_pe"], cfg["n_per_pe"]
        orc.master(cfg, L[0], np.zeros((M, 5)))
    for M in (1, 2, 7, 300):
        orc.ring(11, 0, 3, M)
        orc.ring(11, 1, 70, M, orc.MODE_RNA)
    orc.ring_groups(5, 0, 2, 64, 8)
    P = rng.integers(0, 1 << 20, 50).astype(np.uint32)
    orc.nex(P, 4096)
    Q = rng.integers(0, 1000, 300).astype(np.uint32)
    orc.resample(Q, int(Q.sum()) - 1)
    orc.philox(np.arange(16, dtype=np.uint32).reshape(4, 4), np.array([1, 2], np.uint32))
    print("SANITIZED ORACLE OK")
""")


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-std=gnu11", "-shared", "-fPIC",
                    "-o", lib, SRC, "-lm"], check=True)
    env = dict(os.environ, ARNA_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    res = subprocess.run([sys.executable, "-c", DRIVER], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=600)
    assert res.returncode == 0 and "SANITIZED ORACLE OK" in res.stdout, (
        res.stdout[-2000:] + res.stderr[-4000:])
