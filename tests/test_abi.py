"""The C-ABI library loads, exports every symbol include/ri.h declares, its
structs match the binding's layouts, and argument checks reject bad plans
before touching a device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2207_11336_amd.ri as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             src, flags=re.M):
            if m.group(1) not in ("if", "while", "return", "sizeof"):
                names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = R.load()
    names = _declared_functions()
    assert {"ri_create", "phi_forward", "phi_adjoint", "fb_step", "denoise", "pnp_solve"} <= names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"declared but not exported: {missing}"
    nm = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in nm.splitlines() if " T " in l}
    assert names <= exported
    assert set(R.EXPORTS) <= names


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ri.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu\\n",sizeof(ri_plan_desc),sizeof(ri_solve_opts),'
                   'sizeof(ri_solve_report),sizeof(ri_plan_stats),offsetof(ri_plan_desc,block_offsets),'
                   'offsetof(ri_solve_opts,trace));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(R.ri_plan_desc), ctypes.sizeof(R.ri_solve_opts), ctypes.sizeof(R.ri_solve_report),
            ctypes.sizeof(R.ri_plan_stats), R.ri_plan_desc.block_offsets.offset, R.ri_solve_opts.trace.offset]
    assert got == want


def test_cnn_desc_layout_matches_header(tmp_path):
    src = tmp_path / "szc.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ri_cnn.h"\n'
                   'int main(){printf("%zu %zu\\n",sizeof(ri_cnn_desc),offsetof(ri_cnn_desc,training));}\n')
    exe = tmp_path / "szc"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(R.ri_cnn_desc), R.ri_cnn_desc.training.offset]


@pytest.mark.parametrize("kw,msg", [
    (dict(channels=32), "channels == 64"),
    (dict(layers=2), "layers"),
    (dict(max_h=40), "multiples of 16"),
    (dict(max_batch=0), "CNN"),
])
def test_cnn_create_rejects_bad_descriptions(kw, msg):
    args = dict(layers=10, max_batch=1, max_h=64, max_w=64)
    args.update(kw)
    with pytest.raises(R.RIError) as e:
        R.ri_cnn_create(**args)
    assert e.value.status == R.RI_EINVAL
    assert msg in str(e.value)


@pytest.mark.parametrize("field,value,msg", [
    ("N", 24, "power of two"),
    ("N", 8, "N must be"),
    ("oversample", 3, "oversample"),
    ("kb_support", 5, "kb_support"),
    ("hmax", 6, "hmax"),
    ("n_wplanes", 4, "n_wplanes"),
    ("precision", 16, "precision"),
    ("g_mode", 7, "g_mode"),
    ("tile", 48, "tile"),
])
def test_create_rejects_bad_descriptions(field, value, msg):
    d = R.plan_desc(64, 10)
    setattr(d, field, value)
    uvw = np.zeros((10, 3))
    with pytest.raises(R.RIError) as e:
        R.ri_create(d, uvw)
    assert e.value.status == R.RI_EINVAL
    assert msg in str(e.value)


def test_create_rejects_bad_block_offsets():
    d = R.plan_desc(64, 10, n_blocks=2)
    with pytest.raises(R.RIError) as e:
        R.ri_create(d, np.zeros((10, 3)), block_offsets=np.array([0, 7, 9]))
    assert e.value.status == R.RI_EINVAL


def test_binding_checks_shapes_before_the_call():
    d = R.plan_desc(64, 10)
    with pytest.raises(ValueError):
        R.ri_create(d, np.zeros((11, 3)))
