"""The C-ABI library loads and exports every symbol the header declares
(no GPU calls)."""

import ctypes
import os
import re

import pytest

from paper_1607_06886_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pump.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pump_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpump.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_host_only_calls():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpump.so not built")
    lib = _lib.load()
    assert lib.pump_status_str(0) == b"ok"
    assert lib.pump_status_str(-2) == b"capacity exceeded"
    c = _lib.Config()
    lib.pump_config_default(ctypes.byref(c))
    assert c.n_particles == 128 and c.max_steps == 512 and c.mc_particles == 10000
    assert abs(c.dt - 0.05) < 1e-8 and abs(c.lambda_ - 0.5) < 1e-8
    assert ctypes.sizeof(_lib.Result) % 8 == 0
    # NULL-argument contracts that never reach the device
    assert lib.pump_destroy(None) == 0
    assert lib.pump_plan(None, None, None) == _lib.PUMP_E_ARG
    assert lib.pump_create(None, None, None) == _lib.PUMP_E_ARG


def test_struct_layouts_match_the_header():
    """Field order and sizes of the ctypes mirrors (a mismatch would shift
    every later field)."""
    assert ctypes.sizeof(_lib.AABB) == 24
    assert ctypes.sizeof(_lib.Config) == 96  # 18 four-byte fields, then 3 x int64
    off = {name: getattr(_lib.Problem, name).offset for name, _ in _lib.Problem._fields_}
    assert off["samples"] == 0 and off["n"] == 8 and off["obstacles"] == 16
    assert off["x_init"] == 28 and off["goal"] == 52 and off["alpha"] == 76
    assert off["noise"] == 88 and off["noise_mc"] == 96 and off["mem"] == 104
    assert off["sigma_meas"] == 108 and off["noise_meas"] == 112 and off["noise_mc_meas"] == 120
    assert ctypes.sizeof(_lib.Problem) == 128
    assert _lib.Config.estimator.offset == 60


def test_struct_offsets_agree_with_the_c_compiler(tmp_path):
    """offsetof/sizeof of every field as the host C compiler lays out
    include/pump.h, against the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    structs = {"pump_config": _lib.Config, "pump_problem": _lib.Problem,
               "pump_result": _lib.Result, "pump_batch_tuning": _lib.Tuning}
    rename = {"lambda_": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pump.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            if f == "pad":
                continue
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {rename.get(f, f)}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        cname, f, v = ln.split()
        got[(cname, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            if f != "pad":
                assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
