"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs: it holds none of the factorisation arithmetic and is shared by the
tests, the benchmark and the oracle comparisons. Every batch is reproducible from
(workload, instance, seed). Matrices are returned as float64 numpy arrays; batches as [b, m, n]
(row-major numpy layout of each instance; callers convert to column-major where needed).

Workloads (all FP64, i.i.d. per instance):
  * gaussian:   a_ij ~ N(0, 1)                                             (register-kernel batches)
  * graded:     A = U diag(sigma) V^T with Haar U (m x n), V (n x n) and a prescribed spectrum
                (the paper tests on matrices with prescribed condition numbers, Sections 4-6)
  * kernel:     a_ij = exp(-|x_i - y_j| / 0.1) (exponential covariance, correlation length 0.1 as
                in Section 8.3) or 1/|x_i - y_j|, x_i uniform in [0,1]^2, y_j uniform in
                [2,3] x [0,1] (two unit squares whose centres are 2 apart): numerically low rank
  * gauss_decay: U diag(exp(-(i/w)^2)) V^T with Haar U, V and a width w
Haar matrices are the Q factor of a Gaussian matrix with the sign of diag(R) folded in
(Mezzadri, Notices AMS 2007).
"""
from __future__ import annotations

import os

import numpy as np

SIZES_UNEVEN = (64, 128, 256, 512)


def _rng(seed: int, inst: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(inst), int(stream)]))


def haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """m x n matrix with orthonormal columns, Haar distributed (n <= m)."""
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def gaussian(m: int, n: int, seed: int, inst: int) -> np.ndarray:
    return _rng(seed, inst).standard_normal((m, n))


def graded_sigma_log(n: int, decades: float) -> np.ndarray:
    """sigma_i = 10^(-decades (i-1)/(n-1)), i = 1..n (sigma_1 = 1, sigma_n = 10^-decades)."""
    if n == 1:
        return np.ones(1)
    return 10.0 ** (-decades * np.arange(n) / (n - 1))


def prescribed(m: int, n: int, sigma: np.ndarray, seed: int, inst: int) -> np.ndarray:
    """A = U diag(sigma) V^T with Haar U, V; len(sigma) = min(m, n)."""
    rng = _rng(seed, inst)
    k = min(m, n)
    U = haar(rng, m, k)
    V = haar(rng, n, k)
    return (U * sigma[None, :]) @ V.T


def kernel_points(m: int, n: int, seed: int, inst: int):
    rng = _rng(seed, inst, 1)
    x = rng.random((m, 2))
    y = rng.random((n, 2))
    y[:, 0] += 2.0
    return x, y


def kernel_block(m: int, n: int, seed: int, inst: int, kind: str = "exp", corr: float = 0.1) -> np.ndarray:
    x, y = kernel_points(m, n, seed, inst)
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    if kind == "exp":
        return np.exp(-d / corr)
    if kind == "inv":
        return 1.0 / d
    raise ValueError(kind)


def gauss_decay(m: int, n: int, w: float, seed: int, inst: int) -> np.ndarray:
    k = min(m, n)
    sigma = np.exp(-((np.arange(1, k + 1) / w) ** 2))
    return prescribed(m, n, sigma, seed, inst)


def uneven_shapes(count: int, seed: int, sizes=SIZES_UNEVEN):
    """m, n drawn i.i.d. uniformly from `sizes` (the uneven batch of low-rank blocks)."""
    rng = _rng(seed, 0, 7)
    m = rng.choice(np.asarray(sizes), size=count)
    n = rng.choice(np.asarray(sizes), size=count)
    return m.astype(np.int32), n.astype(np.int32)


# --- batch builders for the named workloads -----------------------------------------------------

def batch_gaussian(batch: int, m: int, n: int, seed: int = 1) -> np.ndarray:
    return np.stack([gaussian(m, n, seed, i) for i in range(batch)])


def batch_graded(batch: int, m: int, n: int, decades: float, seed: int = 2) -> np.ndarray:
    s = graded_sigma_log(min(m, n), decades)
    return np.stack([prescribed(m, n, s, seed, i) for i in range(batch)])


def batch_haar(rng: np.random.Generator, b: int, m: int, n: int) -> np.ndarray:
    """b Haar-distributed m x n matrices with orthonormal columns (batched numpy QR)."""
    G = rng.standard_normal((b, m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.einsum("bii->bi", R))
    d[d == 0] = 1.0
    return Q * d[:, None, :]


def batch_prescribed(batch: int, m: int, n: int, sigma: np.ndarray, seed: int, chunk: int = 2000) -> np.ndarray:
    """batch x (U diag(sigma) V^T) with Haar U (m x k), V (n x k); drawn in chunks from one stream
    per (seed, m, n)."""
    k = min(m, n)
    rng = _rng(seed, m * 100003 + n, 11)
    out = np.empty((batch, m, n))
    for s0 in range(0, batch, chunk):
        c = min(chunk, batch - s0)
        U = batch_haar(rng, c, m, k)
        V = batch_haar(rng, c, n, k)
        out[s0:s0 + c] = np.matmul(U * sigma[None, None, :], np.transpose(V, (0, 2, 1)))
    return out


def kernel_blocks_packed(m, n, seed, kind="exp", corr=0.1, device="cuda", first_inst=0):
    """Kernel blocks for instances first_inst .. first_inst+len(m)-1, evaluated on `device` with
    torch and packed column-major, 256-byte aligned (same layout as pack_colmajor). The points of
    each instance come from the same per-instance host stream as kernel_block(), so a block equals
    kernel_block(m_i, n_i, seed, first_inst + i, kind) up to rounding of the distance evaluation.
    Returns (buffer, element offsets)."""
    import torch
    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    sizes = m * n
    padded = (sizes + 31) // 32 * 32
    offs = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.int64) if len(m) else np.zeros(0, np.int64)
    buf = torch.zeros(int(padded.sum()) if len(m) else 1, dtype=torch.float64, device=device)
    kinds = kind if isinstance(kind, (list, tuple, np.ndarray)) else [kind] * len(m)
    groups = {}
    for i in range(len(m)):
        if kinds[i] is not None:  # None: left zero for the caller to fill
            groups.setdefault((int(m[i]), int(n[i]), kinds[i]), []).append(i)
    for (mm, nn, kd), idx in groups.items():
        for s0 in range(0, len(idx), 512):
            part = idx[s0:s0 + 512]
            X = np.empty((len(part), mm, 2))
            Y = np.empty((len(part), nn, 2))
            for j, i in enumerate(part):
                X[j], Y[j] = kernel_points(mm, nn, seed, first_inst + i)
            Xt = torch.from_numpy(X).to(device)
            Yt = torch.from_numpy(Y).to(device)
            d = torch.sqrt(((Yt[:, :, None, :] - Xt[:, None, :, :]) ** 2).sum(-1))  # [B, n, m]: column-major
            blk = torch.exp(-d / corr) if kd == "exp" else 1.0 / d
            dst = torch.from_numpy(offs[part].astype(np.int64)).to(device)
            cols = torch.arange(mm * nn, device=device)
            buf[(dst[:, None] + cols[None, :]).reshape(-1)] = blk.reshape(-1)
    return buf, offs


def c5_mixture(count, seed, sizes=SIZES_UNEVEN):
    """Shapes, kinds and widths of the mixed batch: m, n uniform on `sizes`; kinds exp / inv /
    gauss_decay in equal thirds in a seeded random order; gauss_decay width w ~ U[4, 64]."""
    m, n = uneven_shapes(count, seed, sizes)
    rng = _rng(seed, 0, 13)
    kinds = np.array(["exp", "inv", "gauss_decay"])[rng.permutation(np.arange(count) % 3)]
    w = rng.uniform(4.0, 64.0, size=count)
    return m, n, kinds, w


def _householder_haar(G):
    import torch
    Qh, Rh = torch.linalg.qr(G)
    d = torch.sign(torch.diagonal(Rh, dim1=-2, dim2=-1))
    d[d == 0] = 1.0
    return Qh * d[:, None, :]


def _orth_haar(G):
    """Q with positive diag(R) of each matrix of the stack G (B x rows x k, rows >= k, FP64): the Q
    factor of a Gaussian matrix normalised this way is Haar distributed. Computed as Cholesky QR
    applied twice (Q = G L^-T with L L^T = G^T G; the second pass restores orthogonality to rounding
    level); any matrix whose Cholesky factorisation fails or whose result is not orthonormal to 1e-13
    is redone by Householder QR with the signs of diag(R) folded into Q (so is the whole stack if a
    library call of the fast path fails)."""
    import torch
    B, _, k = G.shape
    eye = torch.eye(k, dtype=G.dtype, device=G.device)
    try:
        Q = G
        bad = torch.zeros(B, dtype=torch.bool, device=G.device)
        for _ in range(2):
            C = torch.bmm(Q.transpose(1, 2).contiguous(), Q)
            L, info = torch.linalg.cholesky_ex(C)
            bad |= info != 0
            L[bad] = eye
            Linv, info2 = torch.linalg.inv_ex(L)
            bad |= info2 != 0
            Q = torch.bmm(Q, Linv.transpose(1, 2).contiguous())
        E = torch.bmm(Q.transpose(1, 2).contiguous(), Q) - eye
        bad |= ~torch.isfinite(E).all(dim=(1, 2))
        bad |= E.abs().amax(dim=(1, 2)) > 1e-13
    except RuntimeError:
        return _householder_haar(G)
    if bad.any():
        idx = torch.nonzero(bad).flatten()
        Q[idx] = _householder_haar(G[idx])
    return Q


def mixed_blocks_packed(m, n, kinds, w, seed, device="cuda", chunk=64, progress=None):
    """The mixed batch packed column-major (256-byte aligned) on `device`. Kernel blocks as in
    kernel_blocks_packed; gauss_decay blocks U diag(exp(-(i/w)^2)) V^T with Haar U (m x k), V (n x k)
    (orthonormal factors of Gaussian matrices, see _orth_haar), drawn per chunk of `chunk` blocks of
    one (m, n) class (chunks formed in order of w) from a generator seeded by (seed, m, n, chunk);
    chunks of 64 keep the batched LU of the triangular inverses within the BLAS workspace.
    Terms with exp(-(i/w)^2) < 1e-18 (i > 6.44 w) are left out: they change no entry of the block at
    FP64 resolution, and the first k columns of a Haar factor are themselves Haar, so
    k = min(m, n, ceil(6.44 w_max)) per chunk. `progress(text)` is called after each (m, n) class."""
    import torch
    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    kinds = np.asarray(kinds)
    w = np.asarray(w, dtype=np.float64)
    buf, offs = kernel_blocks_packed(m, n, seed, kind=[None if k == "gauss_decay" else str(k) for k in kinds], device=device)
    if progress:
        progress("kernel blocks done")
    gd = np.nonzero(kinds == "gauss_decay")[0]
    groups = {}
    for i in gd:
        groups.setdefault((int(m[i]), int(n[i])), []).append(int(i))
    for (mm, nn), idx in sorted(groups.items()):
        idx = sorted(idx, key=lambda i: (w[i], i))
        for cid, s0 in enumerate(range(0, len(idx), chunk)):
            part = idx[s0:s0 + chunk]
            B = len(part)
            k = int(min(mm, nn, np.ceil(6.44 * w[part].max())))
            gen = torch.Generator(device=device)
            gen.manual_seed((int(seed) * 1000003 + mm * 1009 + nn * 7 + cid * 7919) & 0x7FFFFFFFFFFFFFFF)
            Uh = _orth_haar(torch.randn((B, mm, k), generator=gen, dtype=torch.float64, device=device))
            Vh = _orth_haar(torch.randn((B, nn, k), generator=gen, dtype=torch.float64, device=device))
            ww = torch.from_numpy(w[part]).to(device)
            i1 = torch.arange(1, k + 1, dtype=torch.float64, device=device)
            sig = torch.exp(-((i1[None, :] / ww[:, None]) ** 2))
            # column-major storage of A = (U sigma) V^T is the row-major [n, m] array V (U sigma)^T
            At = torch.bmm(Vh.contiguous(), (Uh * sig[:, None, :]).transpose(1, 2).contiguous())
            dst = torch.from_numpy(offs[part].astype(np.int64)).to(device)
            cols = torch.arange(mm * nn, device=device)
            buf[(dst[:, None] + cols[None, :]).reshape(-1)] = At.reshape(-1)
        if progress:
            progress("gauss_decay %dx%d done (%d blocks)" % (mm, nn, len(idx)))
    return buf, offs
