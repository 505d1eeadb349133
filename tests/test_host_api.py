"""Host-side checks that need no GPU: the library loads and exports every
function include/ddgmres.h declares; argument validation that happens before
any device call; bench.py's single-GPU contract."""
import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddgmres.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:dd_status|void|int|size_t|char\s*\*)\s*\*?\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_paper_path():
    names = declared_functions()
    for n in ["fdfd_op_create", "fdfd_op_apply", "gmres_solve", "gmres_solve_batched",
              "dd_solver_solve", "predict_subspace", "predictor_load", "predictor_destroy",
              "gmres_workspace_bytes", "pca_build", "dd_cnn_train_step", "dd_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1902_00090_amd import _lib
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_operator_argument_validation_on_host():
    from paper_1902_00090_amd import FdfdOp, DDError, _lib
    eps = np.full((10, 10), 2.0, np.float32)
    cases = [dict(omega=-1.0, dx=0.04, npml=2), dict(omega=4.0, dx=0.0, npml=2),
             dict(omega=4.0, dx=0.04, npml=5), dict(omega=float("nan"), dx=0.04, npml=0)]
    for kw in cases:
        with pytest.raises(DDError) as ei:
            FdfdOp(eps, **kw)
        assert ei.value.status == _lib.DD_EINVAL
    with pytest.raises(DDError):
        FdfdOp(np.full((2, 10), 2.0, np.float32), 4.0, 0.04, 0)
    bad = eps.copy()
    bad[3, 3] = np.inf
    with pytest.raises(DDError) as ei:
        FdfdOp(bad, 4.0, 0.04, 2)
    assert ei.value.status == _lib.DD_ENONFINITE
    assert "not finite" in _lib.lib().dd_last_error().decode()


def test_other_entry_points_reject_bad_arguments_on_host():
    from paper_1902_00090_amd import _lib
    lib = _lib.lib()
    h = C.c_void_p()
    assert lib.dd_solver_create(None, 0, None, C.byref(h)) == _lib.DD_EINVAL
    assert lib.dd_cnn_create(30, 16, 1, 10, 1, 0, C.byref(h)) == _lib.DD_EINVAL   # nx % 4 != 0
    assert lib.dd_cnn_create(32, 16, 0, 10, 1, 0, C.byref(h)) == _lib.DD_EINVAL   # max_batch 0
    assert lib.dd_cnn_create(32, 16, 1, 10, 2, 0, C.byref(h)) == _lib.DD_EINVAL   # 2 channels
    assert lib.eim_field(None, 0, None, None, None) == _lib.DD_EINVAL
    assert lib.dd_cnn_predict_eim(None, None, None, 1, None, None) == _lib.DD_EINVAL
    assert lib.predict_subspace(None, None, None, None, 1, None, None) == _lib.DD_EINVAL
    assert lib.pca_build(None, 10, 100, 3, None, None, None) == _lib.DD_EINVAL
    assert lib.proj_loss_batched(None, None, 1, 1, 1, None, None) == _lib.DD_EINVAL
    assert lib.dd_solver_kernel_stats(None, None) == _lib.DD_EINVAL


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_rejects_mismatched_lists_and_subspace_shapes():
    """Per-problem lists of the wrong length and subspaces of the wrong shape
    raise in Python before any pointer array reaches the library (which would
    otherwise read past the end of a short array)."""
    import torch
    from paper_1902_00090_amd import _check_lengths, _check_subspace
    _check_lengths(3, b=[1, 2, 3], x=None, x0=[None, None, None])
    for kw in (dict(b=[1, 2]), dict(x=[1, 2, 3, 4]), dict(x0=[None])):
        with pytest.raises(ValueError):
            _check_lengths(3, **kw)
    D = 40
    assert _check_subspace(None, D) == 0
    assert _check_subspace(torch.zeros((5, D), dtype=torch.complex64), D) == 5
    for bad in (torch.zeros((5, D + 1), dtype=torch.complex64),
                torch.zeros((5 * D,), dtype=torch.complex64),
                torch.zeros((2, 5, D), dtype=torch.complex64),
                torch.zeros((65, D), dtype=torch.complex64)):
        with pytest.raises(ValueError):
            _check_subspace(bad, D)


def _pred_file(path, kind, nx, ny, k, cin, count, payload_bytes):
    import struct
    with open(path, "wb") as f:
        f.write(struct.pack("<8siiiiiiqq", b"DDPRED01", kind, nx, ny, k, cin, 0, count, 0))
        f.write(b"\0" * payload_bytes)


def test_predictor_files_are_checked_on_the_host(tmp_path):
    """predictor_load / dd_cnn_load reject missing, foreign, truncated and
    mismatched files with DD_EINVAL and a message, before touching a device."""
    from paper_1902_00090_amd import _lib
    lib = _lib.lib()
    h = C.c_void_p()
    missing = str(tmp_path / "none.ddp").encode()
    assert lib.predictor_load(missing, 1, C.byref(h)) == _lib.DD_EINVAL
    assert "cannot open" in lib.dd_last_error().decode()
    foreign = tmp_path / "foreign.ddp"
    foreign.write_bytes(b"NOTAPRED" + b"\0" * 100)
    assert lib.predictor_load(str(foreign).encode(), 1, C.byref(h)) == _lib.DD_EINVAL
    assert "not a predictor file" in lib.dd_last_error().decode()
    short = tmp_path / "short.ddp"
    _pred_file(short, 1, 8, 8, 2, 0, 2 * 64, 2 * 64 * 8 - 16)        # 16 bytes missing
    assert lib.predictor_load(str(short).encode(), 1, C.byref(h)) == _lib.DD_EINVAL
    assert "bad header or size" in lib.dd_last_error().decode()
    wrongk = tmp_path / "wrongk.ddp"
    _pred_file(wrongk, 1, 8, 8, 3, 0, 2 * 64, 2 * 64 * 8)             # count != k * D
    assert lib.predictor_load(str(wrongk).encode(), 1, C.byref(h)) == _lib.DD_EINVAL
    pca = tmp_path / "pca.ddp"
    _pred_file(pca, 1, 8, 8, 2, 0, 2 * 64, 2 * 64 * 8)
    assert lib.dd_cnn_load(str(pca).encode(), 1, C.byref(h)) == _lib.DD_EINVAL
    assert "PCA basis" in lib.dd_last_error().decode()
    assert lib.predictor_load(str(pca).encode(), 0, C.byref(h)) == _lib.DD_EINVAL
    n = C.c_size_t(7)
    assert lib.dd_solver_workspace_bytes(None, 1, None, C.byref(n)) == _lib.DD_EINVAL
    assert n.value == 0


@pytest.mark.parametrize("kr", [1, 4, 9])
def test_recycling_small_problem_matches_the_oracle(kr):
    """The host half of subspace recycling (Sec. 1; supplement Sec. 1) on the
    oracle's record of a restarted augmented solve: G = [[I, B], [0, H]] and
    M = W^H S from the last cycle give the same harmonic Ritz values and
    the same span S Z as the oracle's dense generalized eigenproblem, with
    ||A y|| = 1 for every returned column."""
    import workloads as W
    from oracle import fdfd, gmres_aug, recycle
    from paper_1902_00090_amd import harmonic_ritz_host
    rng = np.random.default_rng(kr)
    nx, ny = 10, 8
    eps = (2.085 + 10.165 * (rng.random((ny, nx)) < 0.5)).astype(np.float32)
    inst = W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, 0.04, 1.55, 2)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(rng, (inst.D, 3))
    _, info = gmres_aug.gmres_aug(A, inst.b, V, restart=12, tol=1e-10, maxit=200, record=True)
    S = recycle.last_cycle_space(V, info)
    k, n = 3, info["Q"].shape[1] - 1
    G = np.zeros((k + n + 1, k + n), np.complex128)
    G[:k, :k] = np.eye(k)
    G[:k, k:] = info["B"]
    G[k:, k:] = info["H"]
    Wb = np.concatenate([info["C"], info["Q"]], axis=1)
    M = Wb.conj().T @ S
    Z, th = harmonic_ritz_host(G, M, kr)
    to, Yo = recycle.harmonic_ritz(A, S, kr)
    np.testing.assert_allclose(th, to, rtol=1e-9)
    Y = S @ Z
    np.testing.assert_allclose(np.linalg.norm(A @ Y, axis=0), 1.0, rtol=1e-9)
    Qo, _ = np.linalg.qr(Yo)
    Ql, _ = np.linalg.qr(Y)
    assert np.linalg.norm(Ql - Qo @ (Qo.conj().T @ Ql)) <= 1e-8


def test_recycling_small_problem_rejects_bad_sizes():
    from paper_1902_00090_amd import DDError, harmonic_ritz_host
    G = np.eye(4, 3, dtype=np.complex128)
    with pytest.raises(DDError):
        harmonic_ritz_host(G, G, 4)           # kr > ns
    with pytest.raises(DDError):
        harmonic_ritz_host(np.zeros((4, 3), np.complex128), G, 2)   # rank-deficient G


@pytest.mark.parametrize("seed", range(6))
def test_small_harmonic_ritz_problem_against_generalized_eig(seed):
    """The host eigen-solver of recycling (Householder least squares,
    Hessenberg QR, Schur reordering) on random problems of sizes 1 to 40,
    square and overdetermined: the harmonic Ritz values equal scipy's
    generalized eigenvalues of (G^H G, G^H M) of smallest magnitude, and the
    returned columns span the same invariant subspace with ||G z|| = 1."""
    import scipy.linalg as sla
    from paper_1902_00090_amd import harmonic_ritz_host
    rng = np.random.default_rng(100 + seed)
    ns = int(rng.integers(1, 41))
    nw = ns + int(rng.integers(0, 2))
    kr = int(rng.integers(1, ns + 1))
    G = rng.standard_normal((nw, ns)) + 1j * rng.standard_normal((nw, ns))
    M = rng.standard_normal((nw, ns)) + 1j * rng.standard_normal((nw, ns))
    Z, th = harmonic_ritz_host(G, M, kr)
    w, U = sla.eig(G.conj().T @ G, G.conj().T @ M)
    order = np.argsort(np.abs(w), kind="stable")
    np.testing.assert_allclose(np.sort_complex(th), np.sort_complex(w[order[:kr]]), rtol=1e-8)
    np.testing.assert_allclose(np.linalg.norm(G @ Z, axis=0), 1.0, rtol=1e-10)
    if kr < ns and abs(abs(w[order[kr - 1]]) - abs(w[order[kr]])) > 1e-6 * abs(w[order[kr]]):
        Qa, _ = np.linalg.qr(U[:, order[:kr]])
        Qb, _ = np.linalg.qr(Z)
        assert np.linalg.norm(Qb - Qa @ (Qa.conj().T @ Qb)) <= 1e-7


def test_small_harmonic_ritz_problem_with_repeated_eigenvalues():
    """G = I (square) and M = diag with repeated entries: T = M, whose
    eigenvalues of largest magnitude (smallest 1/theta) come out exactly,
    including a repeated one, and the basis lies in their eigenspace."""
    from paper_1902_00090_amd import harmonic_ritz_host
    d = np.array([1.0, 3.0, 3.0, 0.5, 2.0, 3.0], np.complex128)
    G = np.eye(6, dtype=np.complex128)
    M = np.diag(d)
    Z, th = harmonic_ritz_host(G, M, 3)
    np.testing.assert_allclose(th, 1.0 / 3.0 * np.ones(3), rtol=1e-12)
    # the span is that of e_1, e_2, e_5 (the entries equal to 3)
    P = np.zeros((6, 6))
    P[[1, 2, 5], [1, 2, 5]] = 1.0
    np.testing.assert_allclose(P @ Z, Z, atol=1e-12)
