"""GPU parity of the one-sided block Jacobi (Gram path) of batched_svd."""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05141_amd import synth
from svd_checks import check_svd

pytestmark = pytest.mark.gpu

import paper_1707_05141_amd as P  # noqa: E402
from paper_1707_05141_amd import _lib  # noqa: E402

W_FLAGS = {8: _lib.SVD_BLOCK_W8, 16: _lib.SVD_BLOCK_W16, 32: _lib.SVD_BLOCK_W32}


def _svd(A_np, flags, dtype=torch.float64):
    A = torch.from_numpy(A_np).to(device="cuda", dtype=dtype)
    S, U, V, sw, info = P.svd(A, flags=flags)
    torch.cuda.synchronize()
    return S.double().cpu().numpy(), U.double().cpu().numpy(), V.double().cpu().numpy(), sw.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("m,n,w", [(64, 32, 8), (96, 40, 8), (128, 64, 16), (100, 70, 16), (200, 128, 32), (40, 100, 8),
                                   (130, 96, 32)])
def test_block_vs_oracle(m, n, w):
    print("case: block %dx%d w=%d" % (m, n, w), flush=True)
    A = synth.batch_gaussian(3, m, n, seed=m + n + w)
    S, U, V, sw, info = _svd(A, _lib.SVD_FORCE_BLOCK | W_FLAGS[w])
    So, Uo, Vo, swo, io = oracle.batched_jacobi_svd(A)
    for b in range(3):
        assert info[b] == 0, (b, info[b], sw[b])
        check_svd(A[b], S[b], U[b], V[b], So[b], Uo[b], Vo[b], 1e-12, vec_tol=1e-8, fac_tol=1e-12)


@pytest.mark.parametrize("w", [16, 32])
def test_block_graded_512x256(w):
    """kappa = 1e10 (sigma_i = 10^(-10 (i-1)/255)): the prescribed singular values to 1e-12 sigma_max."""
    print("case: block graded 512x256 w=%d" % w, flush=True)
    sig = synth.graded_sigma_log(256, 10.0)
    A = synth.batch_prescribed(3, 512, 256, sig, seed=7)
    S, U, V, sw, info = _svd(A, _lib.SVD_FORCE_BLOCK | W_FLAGS[w])
    for b in range(3):
        assert info[b] == 0, (sw[b], info[b])
        assert np.max(np.abs(S[b] - sig)) <= 1e-12
        # accumulated block rotations: orthogonality to c * n * m * u in Frobenius norm
        assert np.linalg.norm(V[b].T @ V[b] - np.eye(256)) <= 1e-10
        assert np.linalg.norm(A[b] - (U[b] * S[b]) @ V[b].T) <= 1e-11 * np.linalg.norm(A[b])
        # block rotations from two inner sweeps of G: a few more outer sweeps than with fully
        # converged inner SVDs on this graded spectrum (about 20 at w = 8, 16 at w = 16)
        assert 3 <= sw[b] <= 26
    print("block sweeps", sw)


def test_block_fp32():
    sig = synth.graded_sigma_log(128, 10.0)
    A = synth.batch_prescribed(4, 256, 128, sig, seed=9)
    A32 = A.astype(np.float32).astype(np.float64)
    S, U, V, sw, info = _svd(A, _lib.SVD_FORCE_BLOCK, torch.float32)
    assert np.all(info == 0), (info, sw)
    So = oracle.batched_jacobi_svd(A32, want_vectors=False)[0]
    for b in range(4):
        assert np.max(np.abs(S[b] - So[b])) <= 1e-5 * So[b][0]
        assert np.linalg.norm(A32[b] - (U[b] * S[b]) @ V[b].T) <= 1e-5 * np.linalg.norm(A32[b])


def test_block_auto_route_large():
    """Shapes beyond the register / LDS kernels go to the block path without a flag."""
    A = synth.batch_gaussian(2, 300, 160, seed=3)
    S, U, V, sw, info = _svd(A, 0)
    So, Uo, Vo, _, _ = oracle.batched_jacobi_svd(A)
    for b in range(2):
        assert info[b] == 0
        check_svd(A[b], S[b], U[b], V[b], So[b], Uo[b], Vo[b], 1e-12, vec_tol=1e-8, fac_tol=1e-12)


def test_block_autotuner_picks_and_persists(tmp_path):
    A = synth.batch_gaussian(4, 96, 64, seed=12)
    S, U, V, sw, info = _svd(A, _lib.SVD_FORCE_BLOCK)
    assert np.all(info == 0)
    tuned = P.tune_get(0, 0, 96, 64)
    assert tuned is not None and tuned[0] in (8, 16, 32) and set(tuned[1]) == {8, 16, 32}
    So = oracle.batched_jacobi_svd(A, want_vectors=False)[0]
    np.testing.assert_allclose(S, So, rtol=0, atol=1e-12 * So.max())
    p = tmp_path / "tune.txt"
    P.tune_save(p)
    assert "0 0 96 64 %d" % tuned[0] in p.read_text()
    P.tune_load(p)


def test_tune_cache_load_rejects_unsupported_values(tmp_path):
    """A loaded cache may name the single-kernel path (value 0) for R_B classes up to 128 columns
    only; widths other than 8, 16 and 32 and a 0 above 128 columns are skipped."""
    p = tmp_path / "tune_bad.txt"
    p.write_text("# kind dtype M N value\n1 0 96 96 0\n1 0 480 480 0\n1 0 448 448 12\n0 0 400 300 0\n")
    P.tune_load(p)
    assert P.tune_get(1, 0, 96, 96)[0] == 0
    assert P.tune_get(1, 0, 480, 480) is None
    assert P.tune_get(1, 0, 448, 448) is None
    assert P.tune_get(0, 0, 400, 300) is None
