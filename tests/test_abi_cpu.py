"""Host-only checks of the C-ABI library: every symbol that include/drpf.h declares is
exported, and parameter validation / workspace errors are reported before any GPU call."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drpf.h")


def _lib():
    from paper_2111_04577_amd import binding
    if not os.path.exists(binding.lib_path):
        from paper_2111_04577_amd import build_lib
        build_lib.build()
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drpf_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    B = _lib()
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def _params(**kw):
    B = _lib()
    cfg = W.config("C1")
    p = B.make_params(cfg, 64)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [
    ("nx", 48), ("nx", 2), ("nz", 3), ("ny", 2), ("ny", 6), ("cn", 0.0), ("pe", -1.0),
    ("dt", 0.0), ("s_factor", 0.99), ("theta_bottom_deg", 190.0), ("rho_ratio", 0.0),
    ("precision", 16), ("lz", 0.0),
])
def test_validation_rejects(field, value):
    B = _lib()
    p = _params(**{field: value})
    rc = B.lib().drpf_validate(ctypes.byref(p))
    assert rc == B.DRPF_EINVAL
    assert len(B.lib().drpf_last_error()) > 0


def test_validation_viscoelastic_beta():
    B = _lib()
    p = _params(viscoelastic=1, beta=0.0)
    assert B.lib().drpf_validate(ctypes.byref(p)) == B.DRPF_EINVAL
    p = _params(viscoelastic=1, beta=0.5, wi=0.5)
    assert B.lib().drpf_validate(ctypes.byref(p)) == B.DRPF_OK


def test_validation_polymer_forms():
    B = _lib()
    L = B.lib()
    ok = dict(viscoelastic=1, beta=0.5, wi=0.5)
    for kw, rc in [(dict(constitutive=1), B.DRPF_EINVAL),               # needs viscoelastic
                   (dict(ok, constitutive=2), B.DRPF_EINVAL),
                   (dict(ok, giesekus_alpha=0.6), B.DRPF_EINVAL),
                   (dict(ok, giesekus_alpha=-0.1), B.DRPF_EINVAL),
                   (dict(viscoelastic=1, beta=1.0, wi=0.5, giesekus_alpha=0.2), B.DRPF_EINVAL),
                   (dict(giesekus_alpha=0.2), B.DRPF_EINVAL),
                   (dict(ok, constitutive=1, giesekus_alpha=0.5), B.DRPF_OK),
                   (dict(ok, giesekus_alpha=0.3), B.DRPF_OK)]:
        p = _params(**kw)
        assert L.drpf_validate(ctypes.byref(p)) == rc, kw
    # the adjoint covers the stress form (Oldroyd-B and Giesekus), not the log-conformation form
    nb = ctypes.c_size_t()
    for kw in (dict(ok, constitutive=1), dict(ok, constitutive=1, giesekus_alpha=0.2)):
        p = _params(**kw)
        assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED
    for kw in (ok, dict(ok, giesekus_alpha=0.2)):
        p = _params(**kw)
        assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_OK
    # single resolution: refine 1 or 2 (0 reads as 2); no adjoint; the phase field on the flow grid
    for r, rc in ((3, B.DRPF_EINVAL), (-1, B.DRPF_EINVAL), (0, B.DRPF_OK), (1, B.DRPF_OK)):
        p = _params(refine=r)
        assert L.drpf_validate(ctypes.byref(p)) == rc, r
    p = _params(refine=1)
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED
    f, c = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.drpf_field_elems(ctypes.byref(p), ctypes.byref(f), ctypes.byref(c)) == B.DRPF_OK
    assert f.value == c.value


def test_validation_advection_scheme():
    """advection 0 (central) or 1 (WENO-Z); the adjoint covers the central form only."""
    B = _lib()
    L = B.lib()
    for a, rc in ((2, B.DRPF_EINVAL), (-1, B.DRPF_EINVAL), (0, B.DRPF_OK), (1, B.DRPF_OK)):
        p = _params(advection=a)
        assert L.drpf_validate(ctypes.byref(p)) == rc, a
    nb = ctypes.c_size_t()
    p = _params(advection=1)
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_OK and nb.value > 0


def test_validation_wall_relaxation():
    """d_w >= 0 and finite; the adjoint covers relaxed walls too (on FP64 grids)."""
    B = _lib()
    L = B.lib()
    for d, rc in ((-0.1, B.DRPF_EINVAL), (float("inf"), B.DRPF_EINVAL), (float("nan"), B.DRPF_EINVAL),
                  (0.0, B.DRPF_OK), (0.5, B.DRPF_OK)):
        p = _params(d_w=d)
        assert L.drpf_validate(ctypes.byref(p)) == rc, d
    nb = ctypes.c_size_t()
    p = _params(d_w=0.1)
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_OK and nb.value > 0
    p = _params(d_w=0.1, precision=32)
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED


def test_adjoint_grid_bound():
    """The transposed fine kernels index with 32-bit integers: the largest grid the step
    accepts (coarse 1024x1024x512, fine 2^32 cells) has no adjoint, one fine cell count
    below 2^31 has."""
    B = _lib()
    L = B.lib()
    nb = ctypes.c_size_t()
    big = _params(nx=1024, ny=1024, nz=512, viscoelastic=1, beta=0.5, wi=0.5)
    assert L.drpf_validate(ctypes.byref(big)) == B.DRPF_OK
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(big), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED
    assert b"2^31" in L.drpf_last_error()
    ok = _params(nx=1024, ny=512, nz=512, viscoelastic=1, beta=0.5, wi=0.5)   # 2^31 fine cells
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(ok), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED
    ok = _params(nx=1024, ny=256, nz=512, viscoelastic=1, beta=0.5, wi=0.5)   # 2^30
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(ok), ctypes.byref(nb)) == B.DRPF_OK


def test_validation_walls_and_checks():
    """Wall velocities finite; check_finite_every >= 0; moving walls have an adjoint, and with
    relaxed walls (d_w > 0) a forward step but no adjoint."""
    B = _lib()
    L = B.lib()
    nb = ctypes.c_size_t()
    p = _params()
    p.u_wall_top[0] = float("nan")
    assert L.drpf_validate(ctypes.byref(p)) == B.DRPF_EINVAL
    p = _params(check_finite_every=-1)
    assert L.drpf_validate(ctypes.byref(p)) == B.DRPF_EINVAL
    p = _params(check_finite_every=10)
    assert L.drpf_validate(ctypes.byref(p)) == B.DRPF_OK
    p = _params()
    p.u_wall_bottom[1] = 0.5
    assert L.drpf_validate(ctypes.byref(p)) == B.DRPF_OK
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_OK
    p.d_w = 0.1
    assert L.drpf_validate(ctypes.byref(p)) == B.DRPF_OK
    assert L.drpf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == B.DRPF_EUNSUPPORTED


C_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "drpf.h"
#define OFF(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("drpf_params %zu\n", sizeof(drpf_params));
  OFF(drpf_params, a_ext); OFF(drpf_params, d_w); OFF(drpf_params, u_wall_bottom);
  OFF(drpf_params, u_wall_top); OFF(drpf_params, check_finite_every);
  printf("drpf_state %zu\n", sizeof(drpf_state));
  OFF(drpf_state, step); OFF(drpf_state, theta);
  printf("drpf_adj %zu\n", sizeof(drpf_adj));
  printf("drpf_field_layout %zu\n", sizeof(drpf_field_layout));
  OFF(drpf_field_layout, elems); OFF(drpf_field_layout, arrays); OFF(drpf_field_layout, origin);
  printf("drpf_layout %zu\n", sizeof(drpf_layout));
  OFF(drpf_layout, field); OFF(drpf_layout, state_bytes);
  return 0;
}
"""


def test_ctypes_structs_match_header(tmp_path):
    """Sizes and field offsets of the binding's ctypes structures equal the C compiler's for
    include/drpf.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    B = _lib()
    src = tmp_path / "probe.c"
    src.write_text(C_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                             check=True).stdout.splitlines())
    classes = {"drpf_params": B.Params, "drpf_state": B.State, "drpf_adj": B.Adj,
               "drpf_field_layout": B.FieldLayout, "drpf_layout": B.Layout}
    for key, val in out.items():
        if "." in key:
            cname, field = key.split(".")
            assert getattr(classes[cname], field).offset == int(val), key
        else:
            assert ctypes.sizeof(classes[key]) == int(val), key


def test_sizes_and_workspace_errors():
    B = _lib()
    L = B.lib()
    p = _params()
    f, c = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.drpf_field_elems(ctypes.byref(p), ctypes.byref(f), ctypes.byref(c)) == 0
    assert (f.value, c.value) == (128 * 64, 64 * 32)
    nb = ctypes.c_size_t()
    assert L.drpf_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
    assert nb.value > 8 * f.value
    h = ctypes.c_void_p()
    # no workspace, misaligned, too small: rejected on the host before any device call
    assert L.drpf_init_grid(ctypes.byref(p), None, nb.value, None, ctypes.byref(h)) == B.DRPF_EWORKSPACE
    assert L.drpf_init_grid(ctypes.byref(p), ctypes.c_void_p(0x1008), nb.value, None,
                            ctypes.byref(h)) == B.DRPF_EWORKSPACE
    assert L.drpf_init_grid(ctypes.byref(p), ctypes.c_void_p(0x10000), nb.value - 1, None,
                            ctypes.byref(h)) == B.DRPF_EWORKSPACE
    assert b"too small" in L.drpf_last_error()
    # FP32 needs less
    p32 = _params(precision=32)
    nb32 = ctypes.c_size_t()
    assert L.drpf_workspace_bytes(ctypes.byref(p32), ctypes.byref(nb32)) == 0
    assert nb32.value < nb.value


def test_null_arguments():
    B = _lib()
    L = B.lib()
    assert L.drpf_step(None, None, 1, None) == B.DRPF_EINVAL
    assert L.drpf_validate(None) == B.DRPF_EINVAL
    assert L.drpf_destroy(None) == B.DRPF_OK


def test_product_path_does_not_import_oracle():
    """The package and its sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2111_04577_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.lower(), fn


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises: there is no CPU or Python fallback."""
    B = _lib()
    monkeypatch.setattr(B, "_LIB", None)
    monkeypatch.setattr(B, "lib_path", str(tmp_path / "libdrpf.so"))
    with pytest.raises(RuntimeError, match="not found"):
        B.lib()
