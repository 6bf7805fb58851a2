"""The C-ABI library loads on the host and exports every entry point the
public header declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "minsr.h")
LIB = os.path.join(ROOT, "paper_2608_18065_amd", "libminsr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(minsr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_symbols()
    for n in ("minsr_create_model", "minsr_sample", "minsr_local_energy", "minsr_jacobian",
              "minsr_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_symbol_list_matches_header():
    import paper_2608_18065_amd as pm
    assert sorted(pm.SYMBOLS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_errors_without_device_calls():
    import paper_2608_18065_amd as pm
    lib = pm.lib()
    # invalid descriptors are rejected on the host before any device work
    d = pm.ModelDesc(10, 1, 3, 16, 0, 0, 0, pm.F64, 1, 64, 0)
    h = ctypes.c_void_p()
    rc = lib.minsr_create_model(ctypes.byref(d), ctypes.byref(h))
    assert rc == -1
    assert b"dim" in lib.minsr_last_error()
    d = pm.ModelDesc(10, 1, 1, 48, 0, 0, 0, pm.F64, 1, 64, 0)
    assert lib.minsr_create_model(ctypes.byref(d), ctypes.byref(h)) == -6
    assert lib.minsr_destroy_model(None) == -1


def test_binding_structs_match_header_layout(tmp_path):
    # sizes and field offsets of the ctypes structures equal those of the C
    # header, compiled here with the host C compiler
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no host C compiler")
    import paper_2608_18065_amd as pm
    structs = {"minsr_model_desc": pm.ModelDesc, "minsr_hamiltonian": pm.Hamiltonian,
               "minsr_step_cfg": pm.StepCfg, "minsr_step_state": pm.StepState,
               "minsr_step_out": pm.StepOut, "minsr_adaptive_cfg": pm.AdaptiveCfg}
    cfields = {"minsr_model_desc": ["Lx", "Ly", "dim", "hidden", "complex_head", "marshall",
                                    "zero_mag", "compute_dtype", "init_seed", "max_Ns", "options"],
               "minsr_hamiltonian": ["kind", "pbc", "J", "h", "J2"],
               "minsr_step_cfg": ["Ns", "form", "eta", "lambda", "mu", "pinv_cutoff",
                                  "ckpt_every", "apply_update"],
               "minsr_step_state": ["dev_momentum", "key", "counter", "dev_counter"],
               "minsr_step_out": ["dev_energy", "dev_dtheta", "dev_status", "dev_eloc",
                                  "dev_sigma", "dev_tnorm", "dev_lambda_used"],
               "minsr_adaptive_cfg": ["lambda_mode", "trust_region", "omega", "dev_lambda",
                                      "dev_report"]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#define __HIP_PLATFORM_AMD__ 1",
             '#include "minsr.h"', "int main(void) {"]
    for name, fields in cfields.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in fields:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    r = subprocess.run(["gcc", "-I", inc, "-I", "/opt/rocm/include", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("header does not compile on the host: " + r.stderr[-300:])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for name, S in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(S), name
        cf = cfields[name]
        pf = [f for f, _ in S._fields_]
        assert len(cf) == len(pf), name
        for c, p in zip(cf, pf):
            assert got[(name, c)] == getattr(S, p).offset, (name, c)
