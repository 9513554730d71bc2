"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point declared in include/ite.h, its host-only grid functions
match the oracle, its argument validation rejects bad input before any
device work, and the product-side MPO builders equal the Hamiltonians."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2606_02930_amd as ite
from paper_2606_02930_amd import hamiltonians
from oracle import ed, mpo
from workload import aim_bath

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ite.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ite_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ite.load_library()
    names = _declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # the Python binding covers the same set
    assert set(names) == set(ite._SIGNATURES)


def test_version_and_default_options():
    assert "gfx950" in ite.ite_version()
    o = ite.ite_default_opts()
    assert o.scheme == ite.SCHEME_TRAP and o.krylov_dim == 10 and o.max_cycles == 1 and o.nsweeps == 1
    assert o.shift_mode == ite.SHIFT_TRACK and o.cutoff == 1e-10
    assert o.init_guess == ite.GUESS_B      # Appendix B: b is the initial guess


@pytest.mark.parametrize("args", [(0.01, 100.0, 1.5), (0.01, 1000.0, 1.3), (0.01, 1e4, 1.3), (0.3, 0.5, 7.0)])
def test_loggrid_matches_oracle(args):
    assert np.array_equal(ite.ite_loggrid(*args), ed.loggrid(*args))


def test_panel_grid_matches_oracle():
    for P, n in [(14, 4), (3, 1), (6, 7)]:
        g = ite.ite_panel_grid(64.0, P, n)
        assert np.allclose(g, ed.panel_grid(64.0, P, n), rtol=0, atol=1e-13)


def test_grid_argument_validation():
    lib = ite.load_library()
    n = ctypes.c_int()
    for bad in [(0.0, 1.0, 1.5), (1.0, 0.5, 1.5), (0.1, 1.0, 1.0), (float("nan"), 1.0, 2.0)]:
        assert lib.ite_loggrid(*bad, None, 0, ctypes.byref(n)) == ite.ITE_EINVAL
    assert lib.ite_panel_grid(-1.0, 3, 2, None, 0, ctypes.byref(n)) == ite.ITE_EINVAL
    assert lib.ite_panel_grid(1.0, 0, 2, None, 0, ctypes.byref(n)) == ite.ITE_EINVAL
    # too small a buffer reports the needed count
    buf = (ctypes.c_double * 3)()
    assert lib.ite_loggrid(0.01, 100.0, 1.5, buf, 3, ctypes.byref(n)) == ite.ITE_EINVAL
    assert n.value == 25


def test_null_handles_are_rejected():
    lib = ite.load_library()
    assert lib.ite_ctx_create(0, None, None, None) == ite.ITE_EINVAL
    assert lib.ite_ctx_destroy(None) == ite.ITE_EINVAL
    assert lib.ite_imag_step(None, None, 0.1, None, None) == ite.ITE_EINVAL
    assert lib.ite_measure_energy(None, None, None) == ite.ITE_EINVAL
    assert lib.ite_mps_destroy(None) == ite.ITE_EINVAL
    assert lib.ite_mpo_destroy(None) == ite.ITE_EINVAL
    h = ctypes.c_void_p()
    assert lib.ite_ctx_create(-1, None, None, ctypes.byref(h)) == ite.ITE_EINVAL
    assert lib.ite_last_error(None) == b"NULL context"
    assert lib.ite_mps_sample(None, 4, 3, None, None) == ite.ITE_EINVAL
    # the binding refuses uniforms that are not a [L][nsamples] table before any call
    with pytest.raises(ValueError):
        ite.ite_mps_sample(None, 0, np.zeros(5))


@pytest.mark.parametrize("L", [2, 3, 6])
@pytest.mark.parametrize("Jz", [1.0, 0.0, 0.4])
def test_product_heisenberg_builder_is_the_hamiltonian(L, Jz):
    Ws = hamiltonians.heisenberg(L, J=0.8, Jz=Jz)
    assert [W.shape[:2] for W in Ws][1:-1] == [(5, 5)] * (L - 2)
    H = ed.heisenberg_dense(L, J=0.8, Jz=Jz)
    assert np.abs(mpo.mpo_to_dense(Ws) - H).max() < 1e-14


@pytest.mark.parametrize("nb", [1, 2, 4])
def test_product_anderson_builder_is_the_hamiltonian(nb):
    eb, V = aim_bath(nb, gamma=0.3)
    U = 3.0
    Ws = hamiltonians.anderson_star(U, -U / 2, eb, V)
    assert all(W.shape[2:] == (4, 4) for W in Ws)
    p = ed.aim_basis_permutation(nb + 1)
    Hk = ed.aim_dense(U, -U / 2, eb, V)
    assert np.abs(mpo.mpo_to_dense(Ws) - Hk[np.ix_(p, p)]).max() < 1e-14


def test_product_builders_equal_oracle_builders_as_operators():
    Ws = hamiltonians.heisenberg(5)
    Wo = mpo.heisenberg_mpo(5)
    assert np.abs(mpo.mpo_to_dense(Ws) - mpo.mpo_to_dense(Wo)).max() < 1e-15


def test_bath_grid():
    eb, V = aim_bath(59, 0.1)
    assert len(eb) == 59 and abs(eb[29]) < 1e-15 and np.allclose(eb, -eb[::-1])
    assert np.allclose(V ** 2 * np.pi / (2 / 59), 0.1)


def test_request_footprint_estimate():
    # host-only admission estimate of the serving loop: grows with chi, L and
    # the Krylov dimension, and is bounded by the structurally full bonds
    d8, w8 = [2] * 8, [1] + [5] * 7 + [1]
    f = [ite.ite_request_footprint(d8, w8, chi) for chi in (2, 4, 8, 16)]
    assert all(b > a for a, b in zip(f, f[1:]))
    # L=8 bonds saturate at 2^4 = 16
    assert f[-1] == ite.ite_request_footprint(d8, w8, 32) == ite.ite_request_footprint(d8, w8, 1000)
    assert ite.ite_request_footprint([2] * 64, [1] + [5] * 63 + [1], 256) > \
        ite.ite_request_footprint([2] * 32, [1] + [5] * 31 + [1], 256)
    assert ite.ite_request_footprint(d8, w8, 16, 20) > ite.ite_request_footprint(d8, w8, 16, 10)
    # the c4 maximum (L=128, chi=512) stays within a few GB
    big = ite.ite_request_footprint([2] * 128, [1] + [5] * 127 + [1], 512)
    assert 1e9 < big < 8e9
    assert ite.ite_request_footprint([2], [1, 1], 4) < 0


def test_server_create_validates_options():
    lib = ite.load_library()
    h = ctypes.c_void_p()
    for o in (ite.ite_server_opts(0, 0, 1, 1e9), ite.ite_server_opts(0, 2, 0, 1e9),
              ite.ite_server_opts(0, 2, 1, 0.0)):
        assert lib.ite_server_create(ctypes.byref(o), ctypes.byref(h)) == ite.ITE_EINVAL
    assert lib.ite_server_create(None, ctypes.byref(h)) == ite.ITE_EINVAL


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
def test_gl_coefficients_match_oracle(p):
    # the library's panel coefficients (Newton on the Legendre recurrence,
    # the integrals by the same quadrature) against the oracle's (numpy's
    # Gauss-Legendre rule, polynomial integration of the Lagrange basis)
    from oracle import gauss
    g = ite.ite_gl_coefficients(p)
    c, b, A = gauss.collocation_matrix(p)
    r_inf, w = gauss.end_weights(p)
    assert np.abs(g["c"] - c).max() < 1e-14
    assert np.abs(g["b"] - b).max() < 1e-14
    assert np.abs(g["A"] - A).max() < 1e-12      # the oracle's monomial integration loses ~1e-13 at p = 7
    assert np.abs(g["w"] - w).max() < 1e-11 * max(1.0, np.abs(w).max())
    assert abs(g["r_inf"] - r_inf) < 1e-11 and abs(g["r_inf"] - (-1) ** p) < 1e-11


def test_gl_coefficients_refuse_bad_node_counts():
    lib = ite.load_library()
    buf = (ctypes.c_double * 64)()
    r = ctypes.c_double()
    for p in (0, 8, -1):
        assert lib.ite_gl_coefficients(p, buf, buf, buf, buf, ctypes.byref(r)) == ite.ITE_EINVAL
