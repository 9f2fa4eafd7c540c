"""C-ABI library: it loads, exports every declared symbol, and its host-side
validation rejects invalid arguments without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2605_22281_amd import sfk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfk.h")

pytestmark = pytest.mark.skipif(not os.path.exists(sfk.LIB_PATH), reason="libsfk.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfk_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", sfk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sfk_\w+)", out))
    decl = declared_functions()
    assert decl, "no declarations parsed"
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    assert set(sfk.exported_symbols()) <= exported
    L = sfk.lib()
    for d in decl:
        assert hasattr(L, d)


def test_params_layout_matches_header(tmp_path):
    # sfk_params: 6 int32, uint64 seed, 2 int32, 4 double, 8 int32, perm pointer,
    # 6 int32 and a double of the low-rank operators
    assert ctypes.sizeof(sfk.Params) == 144
    assert sfk.Params.perm.offset == 104 and sfk.Params.lr_tol.offset == 136
    assert sfk.Params.seed.offset == 24 and sfk.Params.eps.offset == 40
    assert ctypes.sizeof(sfk.CSR) == 48
    # the C compiler's layout of the header agrees field by field
    fields = [f[0] for f in sfk.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sfk.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(sfk_params));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(sfk_params, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(sfk.Params)
    assert got[1:] == [getattr(sfk.Params, f).offset for f in fields]


def test_params_perm_requires_int32_device_tensor():
    import torch
    with pytest.raises(ValueError):
        sfk.params(perm=torch.arange(4, dtype=torch.int32))      # host tensor


def test_defaults():
    p = sfk.params()
    assert (p.method, p.ell, p.maxit, p.sketch, p.s, p.zeta) == (0, 2, 50, 0, 101, 8)
    assert p.eta == pytest.approx(1.01)


def _A(m=200, n=80, nnz=500):
    return sfk.host_csr_descriptor(m, n, nnz)


@pytest.mark.parametrize("kw,frag", [
    (dict(ell=-1), "ell"),
    (dict(ell=9), "ell"),
    (dict(s=50, maxit=50), "maxit"),
    (dict(maxit=0), "maxit"),
    (dict(s=3000, maxit=10), "s "),
    (dict(zeta=0), "zeta"),
    (dict(zeta=70, s=90), "zeta"),
    (dict(s=101, maxit=50, sketch="identity"), "identity"),
    (dict(tau="reweight_l1", eps=0.0), "eps"),
    (dict(tol=-1.0), "tol"),
    (dict(noise_norm=float("nan")), "noise"),
    (dict(vw=12), "vw"),
    (dict(vw_b=5), "vw"),
    (dict(resid=3), "resid"),
    (dict(copies=1, vw=1), "copies"),
    (dict(copies=2), "copies"),
    (dict(driver=3), "driver"),
    (dict(method="sflsmr", s=60, maxit=20, noise_norm=1.0), "resid = 2"),
])
def test_validation_rejects(kw, frag):
    p = sfk.params(**kw)
    st, msg = sfk.validate(_A(), None, p)
    assert st == sfk.EINVAL
    assert frag in msg


def test_validation_full_orthogonalisation_methods():
    # sketch, s, zeta and ell do not apply to FLSQR / FLSMR
    for m in ("flsqr", "flsmr"):
        assert sfk.validate(_A(), None, sfk.params(m, maxit=300, s=5, ell=99))[0] == sfk.OK
        assert sfk.validate(_A(), None, sfk.params(m, maxit=1025))[0] == sfk.EINVAL
        assert sfk.validate(_A(), None, sfk.params(m, perm=None, tau="reweight_l1", eps=0))[0] \
            == sfk.EINVAL
    st, msg = sfk.validate(_A(), None, sfk.params("flsmr", noise_norm=1.0))
    assert st == sfk.EINVAL and "resid = 2" in msg
    assert sfk.validate(_A(), None, sfk.params("flsqr", noise_norm=1.0))[0] == sfk.OK
    # workspace of FLSQR grows with maxit (whole bases), not with s
    a = sfk.workspace_bytes(_A(), None, sfk.params("flsqr", maxit=10))
    b = sfk.workspace_bytes(_A(), None, sfk.params("flsqr", maxit=40))
    assert 0 < a < b


def test_validation_accepts_new_options():
    for kw in (dict(resid=1), dict(resid=2), dict(copies=1), dict(vw=0, vw_b=64),
               dict(driver="graph"), dict(method="sflsmr", s=60, maxit=20, noise_norm=1.0, resid=2)):
        assert sfk.validate(_A(), None, sfk.params(**kw))[0] == sfk.OK, kw


def test_validation_dimensions():
    p = sfk.params(s=60, maxit=20)
    assert sfk.validate(_A(0, 10, 0), None, p)[0] == sfk.EINVAL
    assert sfk.validate(_A(100, 80, -1), None, p)[0] == sfk.EINVAL
    B_bad = sfk.host_csr_descriptor(200, 80, 10)          # should be 80 x 200
    st, msg = sfk.validate(_A(), B_bad, p)
    assert st == sfk.EINVAL and "B must be" in msg
    # sparse-sign on m-vectors needs s <= m (sFLSQR); SRHT may pad
    st, _ = sfk.validate(_A(40, 80, 10), None, sfk.params(s=60, maxit=20))
    assert st == sfk.EINVAL
    assert sfk.validate(_A(40, 80, 10), None, sfk.params(s=60, maxit=20, sketch="srht"))[0] == sfk.OK
    assert sfk.validate(_A(), sfk.host_csr_descriptor(80, 200, 10), p)[0] == sfk.OK
    assert sfk.validate(_A(100, 80, 5), None,
                        sfk.params(method="sflsmr", s=80, maxit=20, sketch="identity"))[0] == sfk.OK


def test_workspace_bytes_is_zero_for_invalid_and_grows_with_maxit():
    assert sfk.workspace_bytes(_A(), None, sfk.params(ell=-3)) == 0
    a = sfk.workspace_bytes(_A(), None, sfk.params(s=60, maxit=10))
    b = sfk.workspace_bytes(_A(), None, sfk.params(s=60, maxit=40))
    assert 0 < a < b and a % 256 == 0


def test_last_error_never_null():
    assert isinstance(sfk.lib().sfk_last_error(None), bytes)
    assert "gfx950" in sfk.version()


def test_validation_lowrank_tau():
    A = sfk.host_csr_descriptor(300, 16 * 12, 900)          # unknowns form a 16 x 12 image
    ok = dict(s=60, maxit=20, tau="lowrank", lr_rows=16, lr_rank=4)
    assert sfk.validate(A, None, sfk.params(**ok))[0] == sfk.OK
    assert sfk.validate(A, None, sfk.params(**{**ok, "tau": "lowrank_rnd", "lr_q": 3}))[0] == sfk.OK
    assert sfk.validate(A, None, sfk.params("flsqr", maxit=20, tau="lowrank", lr_rows=16,
                                            lr_rank=4))[0] == sfk.OK
    for kw, frag in [(dict(lr_rows=7), "lr_rows"), (dict(lr_rows=0), "lr_rows"),
                     (dict(lr_rank=12), "lr_rank"), (dict(lr_rank=0), "lr_rank"),
                     (dict(lr_q=17, tau="lowrank_rnd"), "lr_q"), (dict(lr_over=-1), "lr_over"),
                     (dict(lr_tol=float("nan")), "lr_tol"), (dict(driver="graph"), "MULTI"),
                     (dict(lr_maxit=-2), "lr_maxit")]:
        st, msg = sfk.validate(A, None, sfk.params(**{**ok, **kw}))
        assert st == sfk.EINVAL and frag in msg, (kw, msg)
    big = sfk.host_csr_descriptor(300, 200 * 200, 900)
    st, msg = sfk.validate(big, None, sfk.params(**{**ok, "lr_rows": 200, "lr_rank": 50,
                                                     "lr_over": 20}))
    assert st == sfk.EINVAL and "exceed" in msg            # l = 70 > 64 test vectors
    # automatic oversampling is capped at 64 test vectors
    assert sfk.validate(big, None, sfk.params(**{**ok, "lr_rows": 200, "lr_rank": 50}))[0] == sfk.OK
    assert sfk.validate(big, None, sfk.params(**{**ok, "lr_rows": 200, "lr_rank": 40,
                                                 "lr_over": 24}))[0] == sfk.OK
    assert sfk.validate(A, None, sfk.params(**{**ok, "tau": 4}))[0] == sfk.EINVAL
    # the workspace grows by the operator's buffers
    assert sfk.workspace_bytes(A, None, sfk.params(**ok)) > sfk.workspace_bytes(
        A, None, sfk.params(s=60, maxit=20))
