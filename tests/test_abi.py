"""CPU checks of the C ABI: the library loads, exports every entry point that
include/sap.h declares, its structs match the header byte for byte, and
argument validation rejects bad calls before any HIP call is made."""
import ctypes as C
import re
import subprocess
from pathlib import Path

import pytest

import paper_1807_03425_amd as sap

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "sap.h"


def _declared():
    txt = HEADER.read_text()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sap_[A-Za-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "sap_init" in names and "sap_softmin_bwd" in names and len(names) >= 12
    L = C.CDLL(str(sap.LIB_PATH))
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sap._SIGS)


MIRRORED = ("sap_config", "sap_min_result", "sap_info_t", "sap_profile_t", "sap_batch_problem", "sap_pca_info",
            "sap_batch_stats")


def test_struct_layout_matches_header(tmp_path):
    """Every field of every struct the binding mirrors sits at the header's
    offset, and the sizes agree."""
    lines = []
    for name in MIRRORED:
        cls = getattr(sap, name)
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'F({name}, {f})')
    prog = tmp_path / "layout.c"
    body = "\n  ".join(lines)
    prog.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
#define F(T, m) printf("%s.%s %zu\\n", #T, #m, offsetof(T, m));
int main(void) {{
  {body}
  return 0;
}}""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(prog)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                        text=True, check=True).stdout.split("\n") if l)
    for name in MIRRORED:
        cls = getattr(sap, name)
        assert int(out[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def _cfg(**kw):
    base = dict(N=100, n=10, k=3, dtype=sap.SAP_F64, form=sap.SAP_PLAIN, rule=0,
                close_cap=0, alpha=0.01, min_len=0.0, close_d=-1.0)
    base.update(kw)
    return sap.sap_config(**base)


BAD = [
    ("N<2", dict(N=1), 1),
    ("n<1", dict(n=0), 1),
    ("k<1", dict(k=0), 1),
    ("k>n", dict(k=11), 1),
    ("k>16", dict(n=40, k=17), 8),
    ("lds", dict(n=2000, k=8), 8),
    ("dtype", dict(dtype=7), 1),
    ("form", dict(form=3), 1),
    ("rule", dict(rule=2), 1),
    ("alpha<0", dict(alpha=-0.1), 1),
    ("alpha>1", dict(alpha=1.5), 1),
    ("alpha nan", dict(alpha=float("nan")), 1),
    ("min_len<0", dict(min_len=-1.0), 1),
    ("min_len inf", dict(min_len=float("inf")), 1),
    ("close_d nan", dict(close_d=float("nan")), 1),
    ("close_cap<0", dict(close_cap=-5), 1),
    ("cand_cap<0", dict(cand_cap=-1), 1),
    ("cand_cap>128", dict(cand_cap=129), 1),
    ("gemm", dict(gemm=3), 1),
]


@pytest.mark.parametrize("name,kw,status", BAD, ids=[b[0] for b in BAD])
def test_init_rejects_bad_config_before_any_device_call(name, kw, status):
    L = sap.lib()
    h = C.c_void_p(123)
    fake = C.c_void_p(0x1000)            # never dereferenced: validation comes first
    st = L.sap_init(C.byref(_cfg(**kw)), fake, 10 if "n" not in kw else max(kw["n"], 1),
                    fake, None, C.byref(h))
    assert st == status, (name, st, L.sap_last_error(None))
    assert h.value is None
    assert L.sap_last_error(None)


def test_init_rejects_null_pointers_and_short_ldx():
    L = sap.lib()
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert L.sap_init(None, fake, 10, fake, None, C.byref(h)) == 1
    assert L.sap_init(C.byref(_cfg()), None, 10, fake, None, C.byref(h)) == 1
    assert L.sap_init(C.byref(_cfg()), fake, 10, None, None, C.byref(h)) == 1
    assert L.sap_init(C.byref(_cfg()), fake, 10, fake, None, None) == 1
    assert L.sap_init(C.byref(_cfg()), fake, 9, fake, None, C.byref(h)) == 1
    assert b"ldx" in L.sap_last_error(None)


def test_null_handle_calls_fail_cleanly():
    L = sap.lib()
    r = sap.sap_min_result()
    assert L.sap_min_secant(None, C.byref(r)) == 1
    assert L.sap_step(None, None) == 1
    assert L.sap_run(None, 3, None, None, None) == 1
    assert L.sap_destroy(None) == 0


def _batch_call(**kw):
    """sap_batch_run with fake device pointers: argument validation comes
    before any device call."""
    import numpy as np
    L = sap.lib()
    fake = C.c_void_p(0x1000)
    offs = np.array(kw.get("offs", [0, 3]), dtype=np.int64)
    pts = np.array(kw.get("pts", [0, 1, 2]), dtype=np.int32)
    probs = (sap.sap_batch_problem * 1)(sap.sap_batch_problem(kw.get("set", 0), kw.get("k", 2), kw.get("rule", 0),
                                                             0, kw.get("alpha", 0.01)))
    ml = np.array(kw.get("ml", [0.0]), dtype=np.float64)
    return L.sap_batch_run(fake, kw.get("dtype", sap.SAP_F64), kw.get("N", 10), kw.get("n", 4),
                           kw.get("ldx", 4), len(offs) - 1, offs.ctypes.data_as(C.c_void_p),
                           pts.ctypes.data_as(C.c_void_p), ml.ctypes.data_as(C.c_void_p), 1, probs,
                           fake, kw.get("iters", 1), kw.get("cap", 0), fake, fake, None, None, None, None)


BATCH_BAD = [
    ("dtype", dict(dtype=5), 1), ("N<2", dict(N=1), 1), ("n<1", dict(n=0), 1), ("ldx<n", dict(ldx=3), 1),
    ("iters<0", dict(iters=-1), 1), ("cap", dict(cap=200), 1), ("offs0", dict(offs=[1, 3]), 1),
    ("set of 1", dict(offs=[0, 1], pts=[0]), 1), ("point outside X", dict(pts=[0, 1, 10]), 1),
    ("min_len<0", dict(ml=[-1.0]), 1), ("set index", dict(set=1), 1), ("k>n", dict(k=5), 1),
    ("k<1", dict(k=0), 1), ("alpha", dict(alpha=2.0), 1), ("rule", dict(rule=3), 1),
    ("k>16", dict(n=40, ldx=40, k=17), 8), ("lds", dict(n=2000, ldx=2000, k=8), 8),
]


@pytest.mark.parametrize("name,kw,status", BATCH_BAD, ids=[b[0] for b in BATCH_BAD])
def test_batch_rejects_bad_arguments_before_any_device_call(name, kw, status):
    assert _batch_call(**kw) == status, (name, sap.lib().sap_last_error(None))
    assert sap.lib().sap_last_error(None)
