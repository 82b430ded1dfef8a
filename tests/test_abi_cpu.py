"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and its host-side validation follows the documented rules."""
import os
import re

import numpy as np
import pytest

from paper_2409_13344_amd import appga as ap
from paper_2409_13344_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "appga.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:appga_status|const char \*)\s*(appga_\w+)\s*\(", src,
                                 flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return ap.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert not [n for n in names if n != "appga_last_error" and n not in ap._SIGS]


def test_params_default_is_the_papers():
    p = ap.appga_params_default()
    assert p.a == 0.125 and p.b == 1.0 and p.beta == 1.0 and p.eps == 1e-3
    assert p.momentum == ap.APPGA_MOMENTUM_GN and p.precond == ap.APPGA_PRECOND_EM
    ap.appga_validate_params(p)


@pytest.mark.parametrize("field,value", [
    ("lambda1", -1e-3), ("lambda2", -1.0), ("eps", 0.0), ("eps", -1.0), ("omega", 0.0),
    ("omega", 1.5), ("a", 0.0), ("beta", 0.0), ("iterations", -1), ("eps", float("nan")),
    ("gamma_scalar", -0.5),
])
def test_params_domain_errors(field, value):
    p = ap.appga_params_default()
    setattr(p, field, value)
    with pytest.raises(ap.AppgaError) as ei:
        ap.appga_validate_params(p)
    assert ei.value.status == -3


def test_momentum_condition_rules():
    """Lemma 8: omega = 1 needs a < 1/2; b must not equal -a k^omega."""
    p = ap.make_params(omega=1.0, a=0.5)
    with pytest.raises(ap.AppgaError):
        ap.appga_validate_params(p)
    ap.appga_validate_params(ap.make_params(omega=1.0, a=0.49))
    with pytest.raises(ap.AppgaError):
        ap.appga_validate_params(ap.make_params(omega=0.5, a=0.25, b=-0.5))    # t_4 = 0
    ap.appga_validate_params(ap.make_params(omega=0.5, a=0.25, b=-0.3))
    with pytest.raises(ap.AppgaError) as ei:
        ap.appga_validate_params(ap.make_params(momentum=7))
    assert ei.value.status == -1
    with pytest.raises(ap.AppgaError):
        ap.appga_validate_params(ap.make_params(precond=ap.APPGA_PRECOND_FIXED, fixed_p=0.0))


def test_matrix_validation():
    geom = synth.Geometry(8, 12, 16)
    A = synth.siddon_matrix(geom)
    ap.appga_validate_system_matrix(8, 16, 12, A.row_ptr, A.col, A.val)

    def expect(status, **mod):
        rp = mod.get("rp", A.row_ptr)
        col = mod.get("col", A.col)
        val = mod.get("val", A.val)
        n_bins = mod.get("n_bins", 12)
        with pytest.raises(ap.AppgaError) as ei:
            ap.appga_validate_system_matrix(8, 16, n_bins, rp, col, val)
        assert ei.value.status == status

    expect(-2, n_bins=11)                                  # m != n_angles * n_bins
    bad = A.col.copy()
    bad[5] = 64
    expect(-2, col=bad)                                    # column out of range
    bad = A.col.copy()
    bad[5] = -1
    expect(-2, col=bad)
    rp = A.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10] + 0
    rp[10] = rp[11] + 1
    expect(-2, rp=rp)                                      # decreasing row_ptr
    v = A.val.copy()
    v[3] = -0.1
    expect(-3, val=v)                                      # negative value
    v = A.val.copy()
    v[3] = np.nan
    expect(-6, val=v)                                      # non-finite


def test_binding_checks_device_buffer_sizes():
    """The device calls cannot see a buffer's length: the binding checks every tensor
    against the matrix's (m, d) and the session's (B, m, d) before a call reaches the
    library (here the calls never get that far)."""
    torch = pytest.importorskip("torch")
    fake_mat = 0x1234
    ap._MAT_DIMS[fake_mat] = (10, 4)
    try:
        g_ok = torch.zeros((2, 10), dtype=torch.float32)
        with pytest.raises(ValueError, match="g holds 10 elements, needs 20"):
            ap.appga_solve_begin(0, fake_mat, torch.zeros((1, 10)), None, [ap.appga_params_default()] * 2)
        with pytest.raises(ValueError, match="gamma holds"):
            ap.appga_afppa_begin(0, fake_mat, g_ok, torch.zeros((1, 10)), [ap.appga_params_default()] * 2)
        with pytest.raises(ValueError, match="f_init"):
            ap.appga_reconstruct_batch_device(0, fake_mat, g_ok, None, [ap.appga_params_default()] * 2,
                                              torch.zeros(7), torch.zeros(8))
        with pytest.raises(ValueError, match="float32"):
            ap.appga_afppa_batch_device(0, fake_mat, g_ok.double(), None, [ap.appga_params_default()] * 2,
                                        None, torch.zeros(8))
        with pytest.raises(ValueError, match="duals"):
            ap.appga_afppa_batch_device(0, fake_mat, g_ok, None, [ap.appga_params_default()] * 2, None,
                                        torch.zeros(8), torch.zeros(47))
        with pytest.raises(ValueError, match="contiguous"):
            ap.appga_reconstruct_batch_device(0, fake_mat, torch.zeros((10, 2)).t(), None,
                                              [ap.appga_params_default()] * 2, None, torch.zeros(8))
        with pytest.raises(ValueError, match="do not match the matrix"):
            ap.appga_reconstruct_batch(0, fake_mat, 4, np.zeros((2, 10)), np.zeros((1, 10)),
                                       [ap.appga_params_default()] * 2)
        with pytest.raises(ValueError, match="do not match the matrix"):
            ap.appga_afppa_batch(0, fake_mat, 5, np.zeros((2, 10)), None, [ap.appga_params_default()] * 2)
        with pytest.raises(ValueError, match="unknown matrix"):
            ap.appga_solve_begin(0, 0x999, g_ok, None, [ap.appga_params_default()] * 2)
    finally:
        ap._MAT_DIMS.pop(fake_mat, None)
