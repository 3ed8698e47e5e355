"""CPU checks of the seeded input generators (the recipe of the synthetic workloads)."""
import numpy as np
import torch

from paper_1707_05141_amd import synth


def test_mixture_proportions_and_ranges():
    m, n, kinds, w = synth.c5_mixture(3000, seed=5)
    assert set(np.unique(m)) <= {64, 128, 256, 512} and set(np.unique(n)) <= {64, 128, 256, 512}
    cnt = {k: int(np.sum(kinds == k)) for k in ("exp", "inv", "gauss_decay")}
    assert cnt == {"exp": 1000, "inv": 1000, "gauss_decay": 1000}
    assert w.min() >= 4.0 and w.max() <= 64.0
    m2, n2, k2, w2 = synth.c5_mixture(3000, seed=5)
    assert np.array_equal(m, m2) and np.array_equal(kinds, k2) and np.array_equal(w, w2)


def test_mixed_blocks_have_prescribed_structure():
    m, n, kinds, w = synth.c5_mixture(90, seed=7)
    buf, offs = synth.mixed_blocks_packed(m, n, kinds, w, seed=7, device="cpu", chunk=8)
    assert np.all(offs % 32 == 0)  # 256-byte aligned FP64 blocks
    for i in range(len(m)):
        mi, ni = int(m[i]), int(n[i])
        A = buf[int(offs[i]):int(offs[i]) + mi * ni].numpy().reshape(ni, mi).T
        if kinds[i] == "gauss_decay":
            s = np.linalg.svd(A, compute_uv=False)
            ref = np.exp(-((np.arange(1, min(mi, ni) + 1) / w[i]) ** 2))
            np.testing.assert_allclose(s, ref, rtol=0, atol=1e-14)
        else:
            np.testing.assert_allclose(A, synth.kernel_block(mi, ni, 7, i, str(kinds[i])), rtol=1e-13, atol=0)


def test_orth_haar_equals_sign_fixed_householder():
    G = torch.randn((20, 96, 40), dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    Q = synth._orth_haar(G.clone())
    Qh, Rh = torch.linalg.qr(G)
    Qh = Qh * torch.sign(torch.diagonal(Rh, dim1=-2, dim2=-1))[:, None, :]
    assert (Q - Qh).abs().max().item() < 1e-13
