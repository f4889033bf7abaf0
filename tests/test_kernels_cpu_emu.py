"""The library's host code and kernels built for the CPU under the emulation
in tests/cpu_emu (threads as fibers, wave operations as meeting points) with
AddressSanitizer and UndefinedBehaviorSanitizer, and run on the batched-run
shapes.  Catches accesses out of bounds of any
device buffer or LDS block, and wave operations under divergent control flow,
without a GPU.  (The source copies differ from the library's in three
mechanical places: the dynamic LDS declaration, the empty asm statements
that hide values from the optimizer, and the kernel-pointer casts, which here
also register the kernel with the emulated launcher.)"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU = os.path.join(HERE, "cpu_emu")
CSRC = os.path.join(ROOT, "paper_1310_4624_amd", "csrc")


def _prepare(dst):
    os.makedirs(dst)
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    files += [os.path.join(CSRC, "arna.hip"), os.path.join(ROOT, "include", "arna.h")]
    for path in files:
        text = open(path).read()
        text = text.replace("extern __shared__ __align__(16) unsigned char smem[];",
                            "unsigned char *smem = emu_smem();")
        text = re.sub(r'__asm__(?: volatile)?\(""\s*:\s*"\+v"\((\w+)\)\);', r"emu_opaque(\1);", text)
        text = re.sub(r"reinterpret_cast<void \*>\(&(.*)\);", r"emu_reg_ret(&\1);", text)
        assert "__asm__" not in text and "extern __shared__" not in text, path
        open(os.path.join(dst, os.path.basename(path)), "w").write(text)


@pytest.fixture(scope="module")
def checks(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not installed")
    d = tmp_path_factory.mktemp("cpu_emu")
    _prepare(str(d / "src"))
    exe = str(d / "emu_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-w",
           "-I", EMU, "-I", str(d), "-I", str(d / "src"), "-o", exe,
           os.path.join(EMU, "emu_checks.cpp"), os.path.join(EMU, "emu_rt.cpp"), "-lpthread"]
    # the checks program includes src/arna.hip relative to its own directory
    shutil.copy(os.path.join(EMU, "emu_checks.cpp"), str(d / "emu_checks.cpp"))
    cmd[cmd.index(os.path.join(EMU, "emu_checks.cpp"))] = str(d / "emu_checks.cpp")
    subprocess.run(cmd, check=True, timeout=900)
    return exe


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", EMU_THREADS="8")
    res = subprocess.run([exe, *args], env=env, capture_output=True, text=True, timeout=900)
    return res.returncode, res.stderr


@pytest.mark.parametrize("mode", ["0", "1", "2", "3"])
def test_batched_run_in_bounds_and_equal_to_separate_runs(checks, mode):
    # 70 iterations cross the ring-table rebuild at iteration 65
    rc, err = _run(checks, "batch", "70", mode)
    assert rc == 0 and "ALL EQUAL" in err, err[-4000:]


def test_batched_run_with_zeroed_fresh_memory(checks):
    rc, err = _run(checks, "batch", "12", "0", "0")
    assert rc == 0 and "ALL EQUAL" in err, err[-4000:]



def test_trajectory_rows_equal_stepwise_estimates(checks):
    rc, err = _run(checks, "traj")
    assert rc == 0 and "TRAJ EQUAL" in err, err[-4000:]


def test_streaming_kernel_equals_lds_kernel_and_resamples_exactly(checks):
    # PEs of up to 4096 particles: every traced output of the streaming step
    # equals k_step's; 4097..65536 particles per PE: ancestors equal exact
    # systematic resampling of the traced weights
    rc, err = _run(checks, "stream")
    assert rc == 0 and "STREAM EQUAL" in err, err[-4000:]


def test_master_record_kernel_equals_in_kernel_form(checks):
    # k_master loads a thread's log-masses before reducing them; the record
    # is bitwise that of master_block with the same workgroup size
    rc, err = _run(checks, "master")
    assert rc == 0 and "MASTER EQUAL" in err, err[-4000:]
