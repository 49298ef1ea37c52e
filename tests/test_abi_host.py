"""Host-only checks of the C ABI (no device work): exported symbols, struct layouts,
argument validation and error codes of the plan builder."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elfpie.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2209_14671_amd import _lib, build
    if not os.path.exists(build.LIB):
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:elfpie_status|const char\s*\*)\s*(elfpie_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2209_14671_amd import _lib
    assert set(names) == set(_lib.FUNCTIONS)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_layouts_match_the_c_header(tmp_path):
    from paper_2209_14671_amd import _lib
    src = tmp_path / "layout.c"
    fields_p = [f for f, _ in _lib.ProblemC._fields_]
    fields_s = [f for f, _ in _lib.StateC._fields_]
    body = ['#include <stdio.h>', '#include <stddef.h>', '#include "elfpie.h"', 'int main(void){',
            'printf("%zu %zu\\n", sizeof(elfpie_problem), sizeof(elfpie_state));']
    body += [f'printf("%zu\\n", offsetof(elfpie_problem, {f}));' for f in fields_p]
    body += [f'printf("%zu\\n", offsetof(elfpie_state, {f}));' for f in fields_s]
    body += ["return 0;}"]
    src.write_text("\n".join(body))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(_lib.ProblemC) and vals[1] == ctypes.sizeof(_lib.StateC)
    offs_p = [getattr(_lib.ProblemC, f).offset for f in fields_p]
    offs_s = [getattr(_lib.StateC, f).offset for f in fields_s]
    assert vals[2:] == offs_p + offs_s


def problem(**kw):
    from paper_2209_14671_amd import elfpie as E
    case = synth.config_case(1)
    base = dict(n_lo=32, upsample=4, led_k=case.led_k, wavelength_um=0.52, na=0.1, dx_lo_um=1.625)
    base.update(kw)
    return E.Problem(**base)


def ws_status(p):
    from paper_2209_14671_amd import _lib
    lib = _lib.load()
    c, keep = p.to_c()
    n = ctypes.c_size_t(0)
    st = lib.elfpie_workspace_bytes(ctypes.byref(c), ctypes.byref(n))
    return st, int(n.value), lib.elfpie_last_error(None).decode()


def test_defaults_match_the_paper(lib):
    from paper_2209_14671_amd import _lib
    p = _lib.ProblemC()
    assert lib.elfpie_problem_defaults(ctypes.byref(p)) == 0
    assert (p.gamma1, p.gamma2, p.lr, p.alpha, p.beta) == (0.9, 0.999, 1e-2, 1e-3, 1e-3)
    assert p.fidelity == _lib.FID_INTENSITY and p.flags == _lib.PUPIL_SUPPORT


def test_workspace_size_accounts_for_every_buffer(lib):
    from paper_2209_14671_amd import _lib
    st, n, _ = ws_status(problem())
    assert st == 0
    K, S, A, B = 25, 317, 128 * 128, 32 * 32
    assert n >= 2 * K * S * 8 + 3 * A * 8 + K * 8
    st64, n64, _ = ws_status(problem(precision=_lib.F64))
    assert st64 == 0 and n64 > n


@pytest.mark.parametrize("kw,code", [
    (dict(n_lo=512), 3),                       # beyond the largest tile (256^2)
    (dict(n_lo=256, precision=0), 3),          # the 256^2 tile runs in F32 only
    (dict(n_lo=256, led_k=np.zeros((2, 2)), mux=2), 3),  # no multiplexing at 256^2
    (dict(n_lo=48), 3),                        # not a supported size (3 x 16)
    (dict(precision=0, n_lo=128), 3),          # F64 tile of 128^2 does not fit LDS
    (dict(upsample=64), 3),                    # n_hi beyond 1024
    (dict(precision=7), 3),
    (dict(led_k=np.zeros((0, 2))), 1),         # K = 0
    (dict(gamma1=1.0), 1),
    (dict(lr=0.0), 1),
    (dict(alpha=-1.0), 1),
    (dict(fidelity=5), 1),
    (dict(fidelity=2, fid_gamma=0.0), 1),      # x^gamma needs gamma > 0
    (dict(fidelity=2, fid_gamma=5.0), 1),
    (dict(norm=3), 1),
    (dict(flags=64), 1),
    (dict(dx_lo_um=0.0), 1),                   # pixel size must be positive
    (dict(led_k=np.array([[1.0, 0.0]])), 2),   # window far outside the spectrum
    (dict(led_k=np.array([[np.nan, 0.0]])), 1),
])
def test_invalid_problems_are_rejected_before_any_device_work(lib, kw, code):
    st, _, msg = ws_status(problem(**kw))
    assert st == code, msg
    assert msg


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2209_14671_amd import _lib
    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setenv("ELFPIE_LIB", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _lib.load()
    monkeypatch.setattr(_lib, "_LIB", None)


def test_grad_noalloc_rejects_a_problem_larger_than_its_scratch(lib):
    """elfpie_grad_noalloc checks the workspace a problem needs against its 32 MiB static
    scratch on the host, before any device work: 1024^2 / K = 225 / 256^2 needs ~245 MiB."""
    import paper_2209_14671_amd as E
    from paper_2209_14671_amd import _lib
    case = synth.config_case(5)
    prob = E.problem_from_optics(case.optics, case.led_k, precision=E.F32)
    assert E.workspace_bytes(prob) > 32 << 20
    p, _keep = prob.to_c()
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: the call fails first
    st = lib.elfpie_grad_noalloc(ctypes.byref(p), fake, fake, fake, fake, None, None, None)
    assert st == _lib.E_WORKSPACE
    assert b"33554432" in lib.elfpie_last_error(None)
