"""The C interface on the CPU: the library loads, exports every entry point
include/arna.h declares, its structs match the header, and host-side argument
checks reject bad input before any GPU work (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1310_4624_amd import _native as nat
from paper_1310_4624_amd import build as b
from paper_1310_4624_amd.tracker import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "arna.h")


@pytest.fixture(scope="module")
def L():
    if b.stale():
        b.build()
    return nat.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(nat.SIGNATURES), set(names) ^ set(nat.SIGNATURES)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "arna.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(pf_config), sizeof(pf_estimate_t), sizeof(pf_pe_record));
  printf("%zu %zu %zu %zu\\n", offsetof(pf_config, fixed_ratio), offsetof(pf_config, debug),
         offsetof(pf_config, seed), offsetof(pf_config, stream));
  printf("%zu %zu\\n", offsetof(pf_estimate_t, step), offsetof(pf_pe_record, lstar));
  printf("%zu %zu %zu\\n", sizeof(pf_master_t), offsetof(pf_master_t, n_ex),
         offsetof(pf_master_t, step));
  printf("%zu\\n", offsetof(pf_config, pes_per_wg));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(nat.pf_config), ctypes.sizeof(nat.pf_estimate_t),
            ctypes.sizeof(nat.pf_pe_record),
            nat.pf_config.fixed_ratio.offset, nat.pf_config.debug.offset,
            nat.pf_config.seed.offset, nat.pf_config.stream.offset,
            nat.pf_estimate_t.step.offset, nat.pf_pe_record.lstar.offset,
            ctypes.sizeof(nat.pf_master_t), nat.pf_master_t.n_ex.offset, nat.pf_master_t.step.offset,
            nat.pf_config.pes_per_wg.offset]
    assert got == want


def test_strerror_texts(L):
    for code in [0, -1, -2, -3, -4, -5, -6, -7]:
        assert L.pf_strerror(code)
    assert L.pf_strerror(-99) == b"unknown error"


def _init(L, **kw):
    c = make_config(kw, debug=kw.get("debug", 0))
    for k, v in kw.items():
        if k == "struct_size":
            c.struct_size = v
    h = ctypes.c_void_p()
    t = np.zeros((max(1, kw.get("n_filters", 1)), 5), np.float32)
    return L.pf_init(ctypes.byref(c), t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                     ctypes.byref(h))


@pytest.mark.parametrize("bad,code", [
    (dict(n_pe=0), nat.PF_EINVAL),
    (dict(n_per_pe=0), nat.PF_EINVAL),
    (dict(n_filters=0), nat.PF_EINVAL),
    (dict(n_pe=nat.PF_MAX_PE + 1), nat.PF_EUNSUPPORTED),
    (dict(n_per_pe=nat.PF_MAX_PER_PE + 1), nat.PF_EUNSUPPORTED),
    # 17 x 8192 x 4096 > 2^29 particles: 32-bit state indices would wrap
    (dict(n_filters=17, n_pe=nat.PF_MAX_PE, n_per_pe=nat.PF_MAX_PER_PE), nat.PF_EUNSUPPORTED),
    (dict(patch=8), nat.PF_EINVAL),
    (dict(patch=17), nat.PF_EUNSUPPORTED),
    (dict(mode=2), nat.PF_EINVAL),
    (dict(fixed_ratio=1.5), nat.PF_EINVAL),
    (dict(noise_sigma=0.0), nat.PF_EINVAL),
    (dict(psf_sigma=float("nan")), nat.PF_EINVAL),
    (dict(q=-1.0), nat.PF_EINVAL),
    (dict(width=0), nat.PF_EINVAL),
    (dict(struct_size=12), nat.PF_EINVAL),
    (dict(lik_mode=3), nat.PF_EINVAL),
    (dict(lik_mode=nat.PF_LIK_POISSON, background=0.0), nat.PF_EINVAL),
    (dict(ring_groups=257), nat.PF_EINVAL),
    (dict(block_size=100), nat.PF_EINVAL),             # not a multiple of 64
    (dict(block_size=2048), nat.PF_EINVAL),            # above 1024
    (dict(n_per_pe=4096, block_size=512), nat.PF_EINVAL),   # 4 slots per thread do not cover N_p
    # PEs beyond the LDS stage: the streaming kernel's 1024 threads only, and
    # none of lineage tags, multi-iteration launches
    (dict(n_per_pe=5000, block_size=512), nat.PF_EINVAL),
    (dict(n_per_pe=5000, debug=nat.PF_DEBUG_LINEAGE), nat.PF_EUNSUPPORTED),
    (dict(n_per_pe=5000, launch=nat.PF_LAUNCH_PERSISTENT), nat.PF_EUNSUPPORTED),
    # multi-iteration launches take fewer than 2048 PEs
    (dict(n_per_pe=4, n_pe=2048, launch=nat.PF_LAUNCH_PERSISTENT), nat.PF_EUNSUPPORTED),
    # several PEs per workgroup: whole waves per PE, 4 slots per thread at most
    (dict(pes_per_wg=17), nat.PF_EINVAL),
    (dict(n_per_pe=5000, pes_per_wg=2), nat.PF_EINVAL),
    (dict(n_per_pe=256, pes_per_wg=4, block_size=640), nat.PF_EINVAL),   # 160 threads per PE
    (dict(n_per_pe=600, pes_per_wg=8, block_size=1024), nat.PF_EINVAL),  # 128 x 4 < 600
    (dict(n_per_pe=1024, pes_per_wg=16), nat.PF_EINVAL),                 # 64 x 4 < 1024
    (dict(n_per_pe=256, pes_per_wg=4, debug=nat.PF_DEBUG_LINEAGE), nat.PF_EUNSUPPORTED),
    (dict(n_per_pe=256, pes_per_wg=4, launch=nat.PF_LAUNCH_PERSISTENT), nat.PF_EUNSUPPORTED),
])
def test_init_rejects_bad_config_on_host(L, bad, code):
    assert _init(L, **bad) == code


def test_null_arguments_rejected(L):
    assert L.pf_step(None, None) == nat.PF_EINVAL
    assert L.pf_run(None, None, 1, 0) == nat.PF_EINVAL
    assert L.pf_exchange(None, None) == nat.PF_EINVAL
    assert L.pf_estimate(None, None) == nat.PF_EINVAL
    assert L.pf_debug_get(None, 0, None, 0) == nat.PF_EINVAL
    assert L.pf_debug_size(None, 0) == 0
    L.pf_destroy(None)
    assert L.pf_grad_begin(None, 1) == nat.PF_EINVAL
    assert L.pf_grad_end(None, None, 0, None) == nat.PF_EINVAL
    assert L.pf_grad_value(None, None) == nat.PF_EINVAL
    assert L.pf_debug_force_next(None, None, None) == nat.PF_EINVAL
    out = ctypes.c_void_p()
    assert L.pf_batch_create(None, 0, ctypes.byref(out)) == nat.PF_EINVAL
    assert L.pf_batch_run(None, None, None, 1, 0) == nat.PF_EINVAL
    assert L.pf_batch_run_noalloc(None, None, None, 1) == nat.PF_EINVAL
    L.pf_batch_destroy(None)


def test_debug_resample_rejects_bad_offsets_on_host(L):
    q = np.array([[1, 2, 3]], np.uint32)
    anc = np.zeros_like(q)
    v = np.array([6], np.uint32)   # v must be < sum q = 6
    P = ctypes.c_void_p
    assert L.pf_debug_resample_q(P(q.ctypes.data), 1, 3, P(v.ctypes.data),
                                 P(anc.ctypes.data)) == nat.PF_EINVAL
    z = np.zeros((1, 3), np.uint32)
    v0 = np.zeros(1, np.uint32)
    assert L.pf_debug_resample_q(P(z.ctypes.data), 1, 3, P(v0.ctypes.data),
                                 P(anc.ctypes.data)) == nat.PF_EINVAL
    assert L.pf_debug_resample_q(P(q.ctypes.data), 1, 0, P(v.ctypes.data),
                                 P(anc.ctypes.data)) == nat.PF_EINVAL


def test_build_flags_target_gfx950_without_packed_fp32():
    cmds = b.commands("/tmp/x.so", "/tmp")
    assert len(cmds) == 3
    for cmd in cmds[:2]:                      # both translation units
        assert "--offload-arch=gfx950" in cmd
        i = cmd.index("-packed-fp32-ops")
        assert cmd[i - 1] == "-Xclang" and cmd[i - 2] == "-target-feature"
    assert "-disable-machine-licm" in cmds[1] and "-disable-machine-licm" not in cmds[0]
    assert cmds[0][-1].endswith("arna.hip") and cmds[1][-1].endswith("arna_run.hip")
    assert "-shared" in cmds[2]

def test_limit_constants_match_header():
    """The binding's size limits are the header's #defines."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"#define\s+(PF_\w*MAX_\w+)\s+(.+)", text))
    assert set(defs) == {"PF_MAX_PE", "PF_MAX_PER_PE", "PF_MAX_PER_PE_LDS", "PF_MAX_PATCH",
                         "PF_MAX_PARTICLES", "PF_BATCH_NOALLOC_MAX_ARGS"}
    for name, expr in defs.items():
        val = eval(re.sub(r"(\d+)u\b", r"\1", expr.strip()), {})
        assert getattr(nat, name) == val, name
