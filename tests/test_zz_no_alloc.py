"""ppcg_block_pencils_noalloc (scratch in a static device array, for callers
that cannot allocate) against ppcg_block_pencils on the same inputs: equal
bits, on consecutive calls of decreasing size (the second call reuses the
array the first one filled), and the size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dense  # noqa: E402
from paper_1407_7506_amd import binding as B  # noqa: E402


def pencils(nb, nS, cplx, seed):
    rng = np.random.default_rng(seed)
    As, Bs = [], []
    for _ in range(nb):
        M = rng.standard_normal((nS, nS)) + (1j * rng.standard_normal((nS, nS)) if cplx else 0)
        Z = rng.standard_normal((nS, nS)) + (1j * rng.standard_normal((nS, nS)) if cplx else 0)
        Qz, _ = np.linalg.qr(Z)
        As.append(dense.sym(M).T)
        Bs.append(dense.sym((Qz * np.geomspace(1.0, 0.1, nS)) @ Qz.conj().T).T)
    return torch.tensor(np.stack(As), device="cuda"), torch.tensor(np.stack(Bs), device="cuda")


def test_noalloc_pencils_equal_allocating_entry():
    h = B.Handle("fp64")
    # largest first: every later call finds the array holding an earlier call's data
    for q, nb, has_p, cplx, seed in ((32, 20, True, False, 1), (16, 40, True, True, 2), (8, 7, False, False, 3)):
        nS = (3 if has_p else 2) * q
        A, Bm = pencils(nb, nS, cplx, seed)
        C1, f1 = h.block_pencils(A, Bm, q, has_p)
        C2, f2 = h.block_pencils(A, Bm, q, has_p, noalloc=True)
        print("noalloc q", q, "blocks", nb, "P", has_p, "complex", cplx, "flags", f2.cpu().numpy()[:4], flush=True)
        assert torch.equal(C1, C2) and torch.equal(f1, f2)
        assert torch.isfinite(torch.view_as_real(C2) if cplx else C2).all()
    h.close()


def test_noalloc_pencils_reject_oversize():
    h = B.Handle("fp64")
    A, Bm = pencils(100, 96, False, 4)      # 100 pencils of order 96: about 41 MB of scratch
    with pytest.raises(B.PPCGError) as e:
        h.block_pencils(A, Bm, 32, True, noalloc=True)
    assert e.value.status == "PPCG_EINVAL"
    h.close()
