"""Host-side logic without a GPU: the seeded input generators (shapes, ranges,
determinism, the batch recipe), and the measurement helpers of bench.py (the
roofline classification and the rocprofv3 counter reduction)."""
import json
import os
import sqlite3
import sys

import numpy as np
import pytest

from paper_1407_7506_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_default_nbuf_rule():
    for k, q in [(64, 8), (512, 16), (2048, 32), (12, 4), (6, 1), (251, 8)]:
        nb = I.default_nbuf(k, q)
        assert (k + nb) % q == 0
        assert nb >= max(2, int(np.ceil(0.02 * k)))
        assert nb < max(2, int(np.ceil(0.02 * k))) + q


def test_gaussian_wells_range_and_determinism():
    V1 = I.gaussian_wells(16, 0.5, 4, 101)
    V2 = I.gaussian_wells(16, 0.5, 4, 101)
    assert np.array_equal(V1, V2)
    assert V1.shape == (16 ** 3,)
    # sum of 4 wells of depth in (1, 3): never below -12, never positive
    assert V1.max() <= 0 and V1.min() >= -12.0
    assert not np.array_equal(V1, I.gaussian_wells(16, 0.5, 4, 102))


def test_smoothed_field_maps_onto_interval():
    V = I.smoothed_field(12, 0.5, 103)
    assert V.min() == pytest.approx(-2.0) and V.max() == pytest.approx(0.0)


def test_start_block_statistics():
    X = I.start_block(20000, 4, 5)
    assert X.shape == (20000, 4) and X.dtype == np.float64
    assert abs(X.mean()) < 0.02 and abs(X.var() - 1.0) < 0.03
    Z = I.start_block(20000, 4, 5, complex_=True)
    assert Z.dtype == np.complex128
    assert abs(Z.real.var() - 0.5) < 0.02 and abs(Z.imag.var() - 0.5) < 0.02


def test_workload_shapes():
    p = I.wells48()
    assert (p.grid.N, p.grid.order, p.k, p.q, p.K) == (48, 4, 512, 16, 528)
    b = I.bloch96()
    assert (b.grid.N, b.k, b.q, b.K) == (96, 2048, 32, 2112) and b.grid.is_complex
    assert b.grid.kpt[0] == pytest.approx(2 * np.pi * 0.25 / 48.0)
    ps = I.batch64()
    assert len(ps) == 64
    assert all(24 <= p.grid.N <= 40 and 32 <= p.k <= 256 and p.q == 8 and p.K % 8 == 0 for p in ps)
    assert len({(p.grid.N, p.k) for p in ps}) > 40   # uneven sizes


def test_colmajor_roundtrip():
    X = np.arange(12.0).reshape(4, 3)
    B = I.to_colmajor(X)
    assert B.flags["C_CONTIGUOUS"] and B.shape == (3, 4)
    assert np.array_equal(I.from_colmajor(B), X)


def test_roofline_picks_bound_by_intensity():
    # (ms, launches, flops, bytes)
    kt = {"gram_proj": (10.0, 10, 1e12, 1e9), "stencil_f64": (5.0, 10, 1e9, 3e10), "eig": (50.0, 2, 0, 0)}
    r = bench.roofline(kt, "mixed")
    assert r["kernel"] == "gram_proj" and r["bound"] == "mfma" and r["dtype"] == "f32"
    assert r["achieved"] == pytest.approx(100.0)            # 1e12 flops in 10 ms
    assert r["frac"] == pytest.approx(100.0 / 157.3, abs=1e-4)
    kt = {"stencil_f64": (5.0, 10, 1e9, 3e10)}
    r = bench.roofline(kt, "fp64")
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(6000.0) and r["peak"] == 8000.0


def _fake_db(path, counter, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, value real, "
              "counter_name text)")
    c.executemany("insert into counters_collection values (?,?,?,?,?)", [r + (counter,) for r in rows])
    c.commit()
    c.close()


def test_traffic_reduction(tmp_path):
    # the 1 GiB calibration copy reads as 512 MiB (factor 2) and writes as 1 GiB (factor 1)
    gib_kib = float(1 << 20)
    fetch = [(1, "__amd_rocclr_copyBuffer", 1, gib_kib / 2), (2, "__amd_rocclr_copyBuffer", 1, 4.0)]
    write = [(1, "__amd_rocclr_copyBuffer", 1, gib_kib), (2, "__amd_rocclr_copyBuffer", 1, 4.0)]
    # a warmup dispatch (not counted) and two timed ones of the site-1 Gram
    for i, (f, w) in enumerate([(999.0, 999.0), (100.0, 10.0), (300.0, 30.0)]):
        fetch.append((10 + i, "void ppcg::gram_lds_kernel<float, 32, 1>(ppcg::GramArgs)", 256, f))
        write.append((10 + i, "void ppcg::gram_lds_kernel<float, 32, 1>(ppcg::GramArgs)", 256, w))
    fetch.append((20, "void ppcg::gram_kernel<double, 4, 4, false, 0>(ppcg::GramArgs)", 64, 7.0))
    write.append((20, "void ppcg::gram_kernel<double, 4, 4, false, 0>(ppcg::GramArgs)", 64, 7.0))
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _fake_db(fdb, "FETCH_SIZE", fetch)
    _fake_db(wdb, "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    bench.write_traffic(fdb, wdb, {"gram_proj": 2}, "mixed", path=out)
    d = json.load(open(out))
    g = d["kernels"]["gram_proj"]
    assert g["launches"] == 2
    assert g["fetch_bytes_per_launch"] == pytest.approx(2 * 1024 * (100 + 300) / 2, rel=1e-6)
    assert g["write_bytes_per_launch"] == pytest.approx(1024 * (10 + 30) / 2, rel=1e-6)
    assert d["calibration"]["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert d["source_sha"] == bench.kernel_source_sha() and d["precision"] == "mixed"


def test_traffic_kernel_symbols():
    """Each logical kernel of the traffic table matches its device symbols and no other."""
    m = bench._symbol_matches
    gb = bench.TRAFFIC_KERNELS["gram_block"]
    assert m("void ppcg::block_gram_kernel<true, true, true>(ppcg::BlockGramArgs)", *gb)
    assert m("void ppcg::block_gram_kernel<false, false, false>(ppcg::BlockGramArgs)", *gb)
    assert not m("void ppcg::gram_kernel<double, 4, 5, false, 2>(ppcg::GramArgs)", *gb)
    gp = bench.TRAFFIC_KERNELS["gram_proj"]
    assert m("void ppcg::gram_lds_kernel<float, 32, 1>(ppcg::GramArgs)", *gp)
    assert m("void ppcg::gram_kernel<float, 4, 4, false, 1>(ppcg::GramArgs)", *gp)
    assert not m("void ppcg::gram_lds_kernel<double, 16, 0>(ppcg::GramArgs)", *gp)
    up = bench.TRAFFIC_KERNELS["update_proj"]
    assert m("void ppcg::update_lds_kernel<float, 16, 1>(ppcg::UpdateArgs)", *up)
    assert not m("void ppcg::update_lds_kernel<double, 32, 0>(ppcg::UpdateArgs)", *up)


def test_traffic_is_keyed_by_precision(tmp_path, monkeypatch):
    """A counter summary taken on one precision never answers for the other."""
    monkeypatch.setattr(bench, "traffic_path", lambda prec: str(tmp_path / f"t_{prec}.json"))
    d = {"source_sha": bench.kernel_source_sha(), "precision": "mixed",
         "kernels": {"update_proj": {"hbm_bytes_per_launch": 7.0e8}}}
    json.dump(d, open(tmp_path / "t_mixed.json", "w"))
    assert bench.traffic_for("update_proj", "mixed") == 7.0e8
    assert bench.traffic_for("update_proj", "fp64") is None
    json.dump(dict(d, precision="mixed"), open(tmp_path / "t_fp64.json", "w"))
    assert bench.traffic_for("update_proj", "fp64") is None


def test_hbm_rates_and_solve_roofline():
    kt = {"stencil_f64": (10.0, 10, 1e9, 4e10), "gram_proj": (10.0, 10, 1e12, 1e9)}
    r = bench.hbm_rates(kt, "mixed")
    assert list(r) == ["stencil_f64"]                      # the Gram is MFMA-bound by intensity
    assert r["stencil_f64"]["algorithmic_GBps"] == pytest.approx(4000.0)
    sr = bench.solve_roofline({"roofline_ms": 50.0, "time_s": 0.2})
    assert sr["frac"] == pytest.approx(0.25)
    assert bench.stage_ms({"stage_ms": [1, 2, 3, 4, 5, 6]})["cholqr"] == 4


# --- the block-Jacobi round schedule of the Rayleigh-Ritz eigensolver --------
# 16-wide blocks, circle (round-robin) pairing; the device code fuses the pair
# eigensolves of round r with the two-sided update of round r - 1, keeping M_r
# in alternating buffers and forming each pair problem from M_{r-1} and the
# previous round's rotations.  These tests replay that schedule in numpy (the
# pair eigensolves by numpy's eigh) and check it against rounds run one after
# the other, and the inverse of the pairing it relies on.
JB = 16


def _rr_player(pos, rnd, n):
    return 0 if pos == 0 else ((pos - 1 + rnd) % (n - 1)) + 1


def _pair(m, nbe, t, rnd):
    nblk = (m + JB - 1) // JB
    i, j = sorted((_rr_player(t, rnd, nbe), _rr_player(nbe - 1 - t, rnd, nbe)))
    idx = list(range(i * JB, min(m, i * JB + JB))) if i < nblk else []
    return idx + (list(range(j * JB, min(m, j * JB + JB))) if j < nblk else [])


def _locate(nbe, b, rnd):
    n1, npairs = nbe - 1, nbe // 2
    pos = 0 if b == 0 else ((b - 1 - rnd) % n1 + n1) % n1 + 1
    return pos if pos < npairs else nbe - 1 - pos


def _tile(M, Q, rot, a, b, pa, pb):
    T = M[np.ix_(pa, pb)]
    T = T @ Q[b] if rot[b] else T
    return Q[a].T @ T if rot[a] else T


def _sweep_sequential(M, m, nbe):
    M, Vt = M.copy(), np.eye(m)
    for rnd in range(nbe - 1):
        P = [_pair(m, nbe, t, rnd) for t in range(nbe // 2)]
        Q = {t: np.linalg.eigh(M[np.ix_(p, p)])[1] for t, p in enumerate(P) if p}
        rot = {t: bool(p) for t, p in enumerate(P)}
        new = M.copy()
        for a, pa in enumerate(P):
            for b, pb in enumerate(P):
                if pa and pb:
                    new[np.ix_(pa, pb)] = _tile(M, Q, rot, a, b, pa, pb)
        M = new
        for b, pb in enumerate(P):
            if rot[b]:
                Vt[:, pb] = Vt[:, pb] @ Q[b]
    return M, Vt


def _sweep_fused(M, m, nbe):
    home, second, Vt, R = M.copy(), np.full_like(M, np.nan), np.eye(m), nbe - 1
    buf = (lambda r: second if r % 2 else home)
    Qs, rots = [{}, {}], [{}, {}]
    for r in range(R + 1):
        if r < R:  # pair eigensolves of round r, from M_{r-1} and the rotations of r - 1
            par = r & 1
            for t in range(nbe // 2):
                idx = _pair(m, nbe, t, r)
                rots[par][t] = bool(idx)
                if not idx:
                    continue
                if r == 0:
                    S = home[np.ix_(idx, idx)]
                else:
                    prev = [_pair(m, nbe, u, r - 1) for u in range(nbe // 2)]
                    S = np.empty((len(idx), len(idx)))
                    for x, gx in enumerate(idx):
                        for y, gy in enumerate(idx):
                            a, b = _locate(nbe, gx // JB, r - 1), _locate(nbe, gy // JB, r - 1)
                            T = _tile(buf(r - 1), Qs[par ^ 1], rots[par ^ 1], a, b, prev[a], prev[b])
                            S[x, y] = T[prev[a].index(gx), prev[b].index(gy)]
                Qs[par][t] = np.linalg.eigh(S)[1]
        if r >= 1:  # update of round r - 1 into M_r (the caller's matrix after the last round)
            rp, par = r - 1, (r - 1) & 1
            P = [_pair(m, nbe, t, rp) for t in range(nbe // 2)]
            src, dst = buf(rp), (home if rp + 1 == R else buf(rp + 1))
            out = {(a, b): _tile(src, Qs[par], rots[par], a, b, pa, pb)
                   for a, pa in enumerate(P) for b, pb in enumerate(P) if pa and pb}
            for (a, b), v in out.items():
                dst[np.ix_(P[a], P[b])] = v
            for b, pb in enumerate(P):
                if rots[par][b]:
                    Vt[:, pb] = Vt[:, pb] @ Qs[par][b]
    return home, Vt


def test_block_jacobi_pairing_inverse():
    for m in list(range(1, 120)) + [528, 2112]:
        nblk = (m + JB - 1) // JB
        nbe = nblk + (nblk & 1)
        for rnd in range(nbe - 1):
            for t in range(nbe // 2):
                for gx in _pair(m, nbe, t, rnd):
                    assert _locate(nbe, gx // JB, rnd) == t


@pytest.mark.parametrize("m", [17, 40, 48, 70])
def test_fused_jacobi_rounds_equal_sequential_rounds(m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m))
    A = A + A.T
    nblk = (m + JB - 1) // JB
    nbe = nblk + (nblk & 1)
    M1, V1 = _sweep_sequential(A, m, nbe)
    M2, V2 = _sweep_fused(A, m, nbe)
    assert np.array_equal(M1, M2) and np.array_equal(V1, V2)
    # one sweep is a similarity transform by an orthogonal matrix
    assert np.allclose(V1.T @ A @ V1, M1, atol=1e-10)


def test_eig_error_bound_covers_the_true_error():
    """bench.eig_error_bound on a diagonal operator with known spectrum (CPU
    tensors, a stand-in handle): the residuals are those of the Rayleigh
    quotients of perturbed eigenvectors, and the quadratic bound is above
    the true eigenvalue error of every column it covers."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    n, k = 64, 8
    a = np.sort(rng.uniform(1.0, 5.0, n))
    a[:k] = 1.0 + 0.3 * np.arange(k)
    a[k:] += 3.0
    X = np.eye(n)[:, :k] + 1e-4 * rng.standard_normal((n, k))
    X /= np.linalg.norm(X, axis=0)
    lam = np.einsum("ij,i,ij->j", X, a, X)

    class Diag:
        def apply_h(self, V, N, Xcm, h=0.5, order=2):
            return Xcm * torch.tensor(a)[None, :]

    class G:
        N, h, order = 4, 0.5, 2

    r = bench.eig_error_bound(Diag(), None, G(), torch.tensor(lam), torch.tensor(X))
    scale = np.abs(lam).max()
    R = a[:, None] * X - X * lam[None, :]
    assert abs(r["max_col_resid_rel"] - np.linalg.norm(R, axis=0).max() / scale) < 1e-14
    assert r["columns_with_gap"] == k and r["columns"] == k
    assert np.abs(lam - a[:k]).max() / scale <= r["quadratic_bound_rel"]
