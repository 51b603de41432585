"""Host-side checks of the C ABI: exports, status strings and argument validation.

Nothing here launches a kernel; every call below returns before touching the GPU.
"""
import ctypes
import os
import re

import pytest

import paper_1904_11055_amd as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "polyspec.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(polyspec_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ps.load_library()
    names = _declared()
    assert "polyspec_plan" in names and "polyspec_backward" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    assert ps.polyspec_status_string(0) == "ok"
    assert "integral" in ps.polyspec_status_string(5)
    assert ps.polyspec_status_string(99) == "unknown status"


@pytest.mark.parametrize("kw,status", [
    (dict(N=100), 1), (dict(N=16), 1), (dict(N=2048), 1), (dict(order=7), 1), (dict(order=1), 1),
    (dict(n_shells=0), 1), (dict(shell_width=0.0), 1), (dict(shell_width=float("nan")), 1),
    (dict(shell_width=0.1), 1), (dict(batch=0), 1), (dict(precision=3), 1),
    (dict(box_length=-1.0), 1), (dict(flags=1 << 10), 1),
    (dict(n_shells=40), 1),                      # outer edge beyond Nyquist at N = 64
    (dict(n_shells=21), 2),                      # 3 * 21.5 > 64: aliasing without the flag
    (dict(N=512, n_shells=130, shell_width=1.0), 7),  # more shells than the tile kernels hold (128)
    (dict(order=5, N=256, n_shells=40), 7),      # orders 5 and 6 hold at most 32 shells
    (dict(order=6, n_shells=16), 2),             # 6 * 16.5 > 64
])
def test_plan_rejects_bad_descriptors(kw, status):
    args = dict(N=64, order=3, n_shells=16, shell_width=1.0, batch=1, precision=0, box_length=0.0, flags=0)
    args.update(kw)
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_plan(**args)
    assert e.value.status == status
    assert ps.polyspec_last_error(None)


def test_null_arguments():
    lib = ps.load_library()
    assert lib.polyspec_plan(None, None, None) == 1
    assert lib.polyspec_shells(None, None) == 1
    assert lib.polyspec_contract(None, None, None) == 1
    assert lib.polyspec_backward(None, None, None) == 1
    assert lib.polyspec_tuples(None, None, None, None) == 1
    assert lib.polyspec_candidates(None, None, None, None) == 1
    assert lib.polyspec_fields(None, None) == 1
    assert lib.polyspec_workspace_size(None, None) == 1
    assert lib.polyspec_set_workspace(None, None, 0) == 1
    assert lib.polyspec_set_precision(None, 0) == 1
    assert lib.polyspec_destroy(None) == 0


def test_oracle_not_reachable_from_the_package():
    import sys
    import subprocess
    code = ("import sys; import paper_1904_11055_amd as p; p.load_library(); "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert out.stdout.strip() == "False", out.stderr
