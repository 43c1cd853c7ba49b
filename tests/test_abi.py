"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/pasd.h, and validates arguments before touching a GPU."""

import ctypes
import os
import re

import pytest

import paper_1712_09999_amd as pasd
from paper_1712_09999_amd import pasd as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(pasd_[a-z_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = pasd.lib()
    names = _declared()
    assert {"pasd_create", "pasd_step", "pasd_solve", "pasd_destroy"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), name


def _cfg(**kw):
    args = dict(dims=(50, 50, 50), ranks=(5, 5, 5))
    args.update(kw)
    return pasd.make_config(**args)


def test_defaults_follow_algorithm_1():
    c = binding.Config()
    assert pasd.lib().pasd_config_init(ctypes.byref(c)) == 0
    assert (c.mu0, c.mu_max, c.rho, c.tol, c.max_iter) == (1e-4, 1e10, 1.1, 1e-5, 1000)
    assert c.precision == pasd.FP64 and c.device == -1


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(precision="fp32"), 0),
    (dict(dims=(50,), ranks=(5,)), binding.ERR_INVALID_ARG),                  # N < 2
    (dict(ranks=(0, 5, 5)), binding.ERR_INVALID_ARG),                         # R < 1
    (dict(ranks=(51, 5, 5)), binding.ERR_INVALID_ARG),                        # R > I
    (dict(dims=(50, 2, 2), ranks=(5, 2, 2)), binding.ERR_INVALID_ARG),        # R > J
    (dict(dims=(50, 50, 50), ranks=(17, 5, 5)), 0),                           # two rank tiles
    (dict(dims=(100, 100, 100), ranks=(64, 5, 5)), 0),                        # R = 64
    (dict(dims=(100, 100, 100), ranks=(65, 5, 5)), binding.ERR_UNSUPPORTED),  # R > 64
    (dict(dims=(1000, 20, 20), ranks=(9, 5, 5)), 0),                          # tall mode
    (dict(dims=(70000, 4, 4), ranks=(16, 4, 4)), binding.ERR_UNSUPPORTED),   # I R > 2^20
    (dict(dims=(1000, 40, 40), ranks=(17, 5, 5)), binding.ERR_UNSUPPORTED),   # I R > 16384
    (dict(dims=(900, 40, 40), ranks=(18, 5, 5)), 0),                          # I R <= 16384
    (dict(dims=(0, 50, 50)), binding.ERR_INVALID_ARG),
    (dict(lam=(float("nan"), 1, 1)), binding.ERR_INVALID_ARG),
    (dict(mu0=0.0), binding.ERR_INVALID_ARG),
    (dict(mu_max=1e-6), binding.ERR_INVALID_ARG),
    (dict(rho=0.5), binding.ERR_INVALID_ARG),
    (dict(tol=-1.0), binding.ERR_INVALID_ARG),
    (dict(tol=float("nan")), binding.ERR_INVALID_ARG),
    (dict(max_iter=0), binding.ERR_INVALID_ARG),
    (dict(precision=7), binding.ERR_INVALID_ARG),
    (dict(tiebreak="keep"), 0),
])
def test_validation_codes(kw, code):
    assert pasd.validate(_cfg(**kw)) == code
    if code != 0:
        assert binding.last_error() != ""


def test_unknown_flag_rejected():
    c = _cfg()
    c.flags = 8
    assert pasd.validate(c) == binding.ERR_INVALID_ARG
    c.flags = binding.FLAG_NO_GRAPH | binding.FLAG_TIEBREAK_KEEP | binding.FLAG_NO_FLOOR_STOP
    assert pasd.validate(c) == 0


def test_order_above_max_rejected():
    c = _cfg()
    c.order = 9
    assert pasd.validate(c) == binding.ERR_INVALID_ARG


def test_footprint_counts_state():
    c = _cfg()
    b64 = pasd.footprint(c)
    # at least T, D, 3 multipliers and one export buffer of 125 000 doubles
    assert b64 >= 6 * 125000 * 8
    b32 = pasd.footprint(_cfg(precision="fp32"))
    assert b32 < b64
    with pytest.raises(pasd.PasdError):
        pasd.footprint(_cfg(ranks=(0, 5, 5)))


def test_create_rejects_bad_arguments_without_gpu():
    h = ctypes.c_void_p()
    bad = _cfg(ranks=(0, 5, 5))
    buf = (ctypes.c_double * 8)()
    rc = pasd.lib().pasd_create(ctypes.byref(bad), ctypes.cast(buf, ctypes.c_void_p), 0, ctypes.byref(h))
    assert rc == binding.ERR_INVALID_ARG and not h.value
    good = _cfg()
    rc = pasd.lib().pasd_create(ctypes.byref(good), None, 0, ctypes.byref(h))
    assert rc == binding.ERR_INVALID_ARG and not h.value
    pasd.lib().pasd_destroy(None)  # NULL-safe



def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of pasd_config and pasd_info have the C layout: a
    host program compiled from include/pasd.h prints every field's offset and
    the struct sizes, which must equal what ctypes computes."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pasd_config": binding.Config, "pasd_info": binding.Info}
    fields = {name: [f[0] for f in cls._fields_] for name, cls in structs.items()}
    c_name = {"lambda_": "lambda"}  # a Python keyword in the binding
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pasd.h"', "int main(void) {"]
    for name, fl in fields.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in fl:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {c_name.get(f, f)}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    assert len(got) == sum(len(v) for v in fields.values()) + len(structs)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f in fields[name]:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
