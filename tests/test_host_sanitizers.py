"""AddressSanitizer and UndefinedBehaviorSanitizer build of the host plan
compiler (tenso_host.cpp with g++, kernel launchers stubbed): tree builders,
generator tables and the device-free plan compiler run on the workloads' own
term tables (train, binary and ternary trees, ps1 and ps2, FP32 and FP64) and
on a deterministic fuzz of malformed trees and generators.  Any invalid memory
access, leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"


def _write_table(path, inst, n_ary, rank):
    from paper_2603_17711_amd.heom import heom_table
    table, dims = heom_table(inst.H, inst.baths, inst.depth)
    coef, slot, nfac, fend, mats = table.arrays()
    lines = [f"{inst.M} {len(dims)} {n_ary} {rank}", " ".join(map(str, dims)), str(len(coef))]
    mo, fo = 0, 0
    for m in range(len(coef)):
        lines.append(f"{float(coef[m].real)!r} {float(coef[m].imag)!r} {slot[m]} {nfac[m]}")
        for _ in range(nfac[m]):
            e = int(fend[fo])
            d = inst.M if e < 2 else dims[e - 2]
            vals = mats[mo:mo + d * d]
            lines.append(f"{e} {d} " + " ".join(f"{float(v.real)!r} {float(v.imag)!r}" for v in vals))
            mo += d * d
            fo += 1
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def test_plan_compiler_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(f"{ROCM}/lib/libamdhip64.so"):
        pytest.skip("g++ or the HIP runtime is missing")
    exe = tmp_path / "driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           os.path.join(ROOT, "paper_2603_17711_amd", "csrc", "tenso_host.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    tables = []
    cases = [(workloads.spin_boson_train(), 1, 8), (workloads.exciton_7site(), 2, 16),
             (workloads.structured_bath_ternary(), 3, 4)]
    cases += [(inst, 2, inst.rank) for inst in workloads.uneven_batch(n_inst=6, seed=2)]
    for k, (inst, n_ary, rank) in enumerate(cases):
        p = tmp_path / f"table{k}.txt"
        _write_table(str(p), inst, n_ary, rank)
        tables.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)] + tables, capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failed checks" in r.stdout
