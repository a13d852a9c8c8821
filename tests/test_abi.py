"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pn.h declares, validates arguments on the host and
carries the same coupling table as the oracle."""
import ctypes as C
import os
import re

import pytest

from oracle.couplings import coupling_list

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pn_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1807_00410_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared("pn.h")
    assert "pn_setup" in names and "pn_solve" in names and "pn_apply" in names
    nn = _declared("pn_nn.h")
    assert "pn_nn_conv3d" in nn and "pn_net_train_step" in nn
    from paper_1807_00410_amd import _lib as L
    bound = {s[0] for s in L.SIGNATURES + L.NN_SIGNATURES}
    for n in names + nn:
        assert hasattr(lib, n), n
        assert n in bound, n  # the Python binding declares it too


def test_abi_version(lib):
    assert lib.pn_abi_version() == 1


def test_compiled_couplings_equal_oracle_quadrature():
    from paper_1807_00410_amd.solver import coupling_table
    for order in range(1, 8):
        t = {(k, d, kp): v for k, d, kp, v in coupling_table(order)}
        o = {(k, d, kp): v for k, d, kp, v in coupling_list(order)}
        assert set(t) == set(o)
        for key in t:
            assert abs(t[key] - o[key]) < 1e-13


def test_setup_rejects_bad_arguments_on_host(lib):
    from paper_1807_00410_amd import _lib as L
    ctx = C.c_void_p()
    grid = L.PnGrid(4, 4, 4, 0.0, 0)
    med = L.PnMedium(C.c_void_p(16), C.c_void_p(16), 0.0, 0.0)
    assert lib.pn_setup(0, C.byref(grid), C.byref(med), None, C.byref(ctx)) == L.PN_ERR_ARG
    assert lib.pn_setup(8, C.byref(grid), C.byref(med), None, C.byref(ctx)) == L.PN_ERR_ARG
    assert lib.pn_setup(3, None, C.byref(med), None, C.byref(ctx)) == L.PN_ERR_ARG
    bad = L.PnGrid(0, 4, 4, 0.0, 0)
    assert lib.pn_setup(3, C.byref(bad), C.byref(med), None, C.byref(ctx)) == L.PN_ERR_ARG
    badbc = L.PnGrid(4, 4, 4, 0.0, 7)
    assert lib.pn_setup(3, C.byref(badbc), C.byref(med), None, C.byref(ctx)) == L.PN_ERR_ARG
    nulls = L.PnMedium(None, None, 0.0, 0.0)
    assert lib.pn_setup(3, C.byref(grid), C.byref(nulls), None, C.byref(ctx)) == L.PN_ERR_ARG
    badg = L.PnMedium(C.c_void_p(16), C.c_void_p(16), 1.5, 0.0)
    assert lib.pn_setup(3, C.byref(grid), C.byref(badg), None, C.byref(ctx)) == L.PN_ERR_ARG
    assert b"g must be" in lib.pn_last_error(None)
    assert lib.pn_setup(3, C.byref(grid), C.byref(med), None, None) == L.PN_ERR_ARG
    assert ctx.value is None
    # null context calls
    assert lib.pn_apply(None, None, None, 0) == L.PN_ERR_ARG
    assert lib.pn_solve(None, None, None, 1e-8, None, None) == L.PN_ERR_ARG
    assert lib.pn_row_weights(None, None) == L.PN_ERR_ARG
    ms = C.c_double()
    assert lib.pn_bench_kernel(None, 0, 1, C.byref(ms)) == L.PN_ERR_ARG
    lib.pn_destroy(None)


def test_status_strings(lib):
    assert lib.pn_status_string(0) == b"ok"
    assert lib.pn_status_string(5) == b"not converged"


def test_batch_setup_rejects_bad_arguments_on_host(lib):
    from paper_1807_00410_amd import _lib as L
    b = C.c_void_p()
    probs = (L.PnProblem * 1)()
    assert lib.pn_batch_setup(0, probs, 1, 0, None, C.byref(b)) == L.PN_ERR_ARG
    assert lib.pn_batch_setup(1, probs, 0, 0, None, C.byref(b)) == L.PN_ERR_ARG
    assert lib.pn_batch_setup(1, None, 1, 0, None, C.byref(b)) == L.PN_ERR_ARG
    assert lib.pn_batch_setup(1, probs, 1, 0, None, None) == L.PN_ERR_ARG
    assert lib.pn_batch_last_error(None)
    assert lib.pn_batch_solve(None, None, None, 1e-8, None, None) == L.PN_ERR_ARG
    assert lib.pn_batch_unknowns(None) == -1
    assert lib.pn_batch_zchunk(None, 0) == -1
    lib.pn_batch_destroy(None)


def test_tune_cache_file_roundtrip_on_host(lib, tmp_path):
    from paper_1807_00410_amd import _lib as L
    lib.pn_tune_cache_clear()
    src = tmp_path / "in.txt"
    src.write_text("# comment\n5 128 128 128 0 5 0.2\n3 64 64 64 1 8 0.01\n")
    assert lib.pn_tune_cache_load(str(src).encode()) == L.PN_OK
    assert lib.pn_tune_cache_size() == 2
    out = tmp_path / "out.txt"
    assert lib.pn_tune_cache_save(str(out).encode()) == L.PN_OK
    rows = sorted(l.split()[:6] for l in out.read_text().splitlines() if not l.startswith("#"))
    assert rows == [["3", "64", "64", "64", "1", "8"], ["5", "128", "128", "128", "0", "5"]]
    bad = tmp_path / "bad.txt"
    bad.write_text("5 128 128 0 5 0.2\n")
    assert lib.pn_tune_cache_load(str(bad).encode()) == L.PN_ERR_ARG
    assert lib.pn_tune_cache_load(str(tmp_path / "missing.txt").encode()) == L.PN_ERR_ARG
    assert lib.pn_autotune(None, 3, None, None) == L.PN_ERR_ARG
    lib.pn_tune_cache_clear()
    assert lib.pn_tune_cache_size() == 0


def test_net_rejects_bad_arguments_on_host(lib):
    from paper_1807_00410_amd import _lib as L
    assert lib.pn_net_nparams() == 15 * (27 * 32 * 32 + 32)
    assert lib.pn_net_create(0, None, None) == L.PN_ERR_ARG
    assert lib.pn_net_forward(None, 1, 8, 8, 8, None, None) == L.PN_ERR_ARG
    assert lib.pn_nn_conv3d(0, 8, 8, 8, None, None, None, 0, 0, None, None) == L.PN_ERR_ARG
    assert lib.pn_nn_pool2(1, 7, 8, 8, C.c_void_p(16), C.c_void_p(16), None) == L.PN_ERR_ARG
    assert lib.pn_nn_adam(None, None, None, None, 10, 1, 1e-3, 0.9, 0.999, 1e-8, None) == L.PN_ERR_ARG
    assert lib.pn_nn_last_error()
    lib.pn_net_destroy(None)


def test_row_weight_constant_matches_assembled_interior_rows():
    # The equilibrated variant weights row k by 1 / (d^2 + c_k / h^2), c_k
    # twice the sum of the squared couplings of row k in the compiled table.
    # Away from the boundary that is the squared 2-norm of the oracle's
    # assembled row: check c_k / h^2 = ||row||^2 - d^2 there.
    import numpy as np
    from oracle.assemble import assemble
    from paper_1807_00410_amd.solver import coupling_table
    rng = np.random.default_rng(4)
    for order in (1, 2, 3, 5):
        dims = (6, 5, 7)
        shp = (dims[2], dims[1], dims[0])
        st = rng.uniform(1.0, 30.0, shp).astype(np.float32)
        al = rng.uniform(0.3, 0.95, shp).astype(np.float32)
        A, lay = assemble(order, dims, st, al, 0.4, 0.5)
        A = A.tocsr()
        h = 1.0 / dims[0]
        ck = {}
        for k, d, kp, v in coupling_table(order):
            ck[k] = ck.get(k, 0.0) + 2.0 * v * v
        rn2 = np.asarray(A.multiply(A).sum(axis=1)).ravel()
        off2 = rn2 - A.diagonal() ** 2
        nnz = np.diff(A.indptr)
        for k in range(len(lay.offset) - 1):
            sl = slice(lay.offset[k], lay.offset[k + 1])
            full = nnz[sl] == nnz[sl].max()
            assert full.any()
            assert np.allclose(off2[sl][full], ck[k] / h ** 2, rtol=1e-12, atol=0.0)
