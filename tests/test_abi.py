"""C ABI checks that need no GPU: the library loads, exports every function
include/fepll.h declares, and rejects invalid arguments before touching the
device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import fepll_synth as fs
import paper_1710_08124_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fepll.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fepll_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared()
    assert "fepll_restore" in names and "fepll_gmm_create" in names
    out = subprocess.run(["nm", "-D", "--defined-only", F.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = F.lib()
    for n in names:
        getattr(L, n)


def test_struct_layouts_match_header(tmp_path):
    """The binding's structs against the C compiler's layout of the header
    (sizes and every field offset)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    fields = {"fepll_image": F.Image, "fepll_options": F.Options, "fepll_tuning": F.Tuning,
              "fepll_operator": F.Operator}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fepll.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, py in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_options_defaults_and_version():
    o = F.Options()
    F.lib().fepll_options_default(ctypes.byref(o))
    assert (o.precision, o.recheck, o.use_proposal, o.top_m) == (0, 1, 0, 8)
    assert o.margin_nats == 0.5
    assert F.lib().fepll_version().decode().startswith("fepll")


def _create(U, lam, w, d=64):
    h = ctypes.c_void_p()
    st = F.lib().fepll_gmm_create(U.ctypes.data, lam.ctypes.data, w.ctypes.data, w.shape[0], d,
                                  ctypes.byref(h))
    return st, h


@pytest.fixture(scope="module")
def gmm3():
    return fs.gmm(3, 1)


def test_create_rejects_wrong_dimension(gmm3):
    U, lam, w = gmm3
    st, h = _create(U, lam, w, d=49)
    assert st == -1 and not h.value
    assert b"64" in F.lib().fepll_last_error()


def test_create_rejects_bad_weights(gmm3):
    U, lam, w = gmm3
    st, _ = _create(U, lam, w * 1.01)
    assert st == -1 and b"sum" in F.lib().fepll_last_error()
    w2 = w.copy()
    w2[0] = -w2[0]
    assert _create(U, lam, w2)[0] == -1
    w3 = w.copy()
    w3[1] = np.nan
    assert _create(U, lam, w3)[0] == -1


def test_create_rejects_bad_eigenvalues(gmm3):
    U, lam, w = gmm3
    l2 = lam.copy()
    l2[1, 5] = -1.0
    assert _create(U, l2, w)[0] == -1
    l2[1, 5] = np.inf
    assert _create(U, l2, w)[0] == -1


def test_create_rejects_non_orthonormal_basis(gmm3):
    U, lam, w = gmm3
    U2 = U.copy()
    U2[2, 3, 4] += 1e-6
    st, _ = _create(U2, lam, w)
    assert st == -1 and b"orthonormal" in F.lib().fepll_last_error()


def test_create_rejects_K_out_of_range():
    U, lam, w = fs.gmm(1, 2)
    h = ctypes.c_void_p()
    assert F.lib().fepll_gmm_create(U.ctypes.data, lam.ctypes.data, w.ctypes.data, 0, 64,
                                    ctypes.byref(h)) == -1
    assert F.lib().fepll_gmm_create(None, lam.ctypes.data, w.ctypes.data, 1, 64,
                                    ctypes.byref(h)) == -1


def test_restore_rejects_null_handle():
    y = np.zeros((16, 16), np.float32)
    yi = F._image(y)
    oi = F._image(np.zeros_like(y))
    st = F.lib().fepll_restore(None, ctypes.byref(yi), None, 10.0, None, 0, ctypes.byref(oi),
                               None, None)
    assert st == -1


def test_batch_and_tuning_reject_bad_arguments():
    y = np.zeros((16, 16), np.float32)
    yi = (F.Image * 1)(F._image(y))
    oi = (F.Image * 1)(F._image(np.zeros_like(y)))
    sg = np.array([10.0])
    L = F.lib()
    assert L.fepll_restore_batch(None, 1, yi, sg.ctypes.data, oi, None) == -1
    t = F.Tuning(768, 4096, 32, 0)
    assert L.fepll_set_tuning(None, ctypes.byref(t)) == -1
    assert L.fepll_get_tuning(None, ctypes.byref(t)) == -1
    assert L.fepll_autotune(None, 1, yi, sg.ctypes.data, None, None) == -1
    assert L.fepll_gmm_flat_tail(None, 0.9, None) == -1


def test_cov_eig_matches_numpy():
    """The library's float64 Jacobi eigendecomposition (host only) against
    numpy.linalg.eigh: same spectrum, orthonormal U, U diag(lam) U^t = Sigma,
    decreasing order."""
    rng = np.random.default_rng(9)
    K, d = 3, 64
    A = rng.standard_normal((K, d, d))
    Sigma = A @ A.transpose(0, 2, 1) * 10.0
    Sigma[2] = Sigma[2] / 1e6 + np.eye(d)  # a near-isotropic one
    U, lam = F.cov_eig(Sigma)
    for k in range(K):
        want = np.sort(np.linalg.eigvalsh(Sigma[k]))[::-1]
        np.testing.assert_allclose(lam[k], want, rtol=1e-10, atol=1e-10 * want[0])
        assert np.all(np.diff(lam[k]) <= 0)
        np.testing.assert_allclose(U[k].T @ U[k], np.eye(d), atol=1e-12)
        np.testing.assert_allclose(U[k] @ np.diag(lam[k]) @ U[k].T, Sigma[k],
                                   atol=1e-11 * np.abs(Sigma[k]).max())


def test_cov_eig_recovers_the_synthetic_mixture():
    U0, lam0, _ = fs.gmm(4, 3)
    Sigma = U0 @ (lam0[:, :, None] * U0.transpose(0, 2, 1))
    U, lam = F.cov_eig(Sigma)
    np.testing.assert_allclose(lam, lam0, rtol=1e-11, atol=1e-9)
    # eigenvectors up to sign (the spectra have distinct eigenvalues)
    sgn = np.sign(np.sum(U * U0, axis=1))
    np.testing.assert_allclose(U * sgn[:, None, :], U0, atol=1e-9)


def test_cov_eig_rejects_bad_input():
    d = 64
    S = np.eye(d)[None].copy()
    S[0, 1, 2] = 0.5  # not symmetric
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.cov_eig(S)
    S = -np.eye(d)[None]  # negative definite
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.cov_eig(S)
    S = np.eye(d)[None].copy()
    S[0, 3, 3] = np.nan
    with pytest.raises(F.FepllError, match="EINVAL"):
        F.cov_eig(S)
