"""GPU parity of the unstructured-midpoint filter (topo_edm_*) with the
oracle: the CSR weight matrix against the oracle's sparse distance weights
(eq. filter_cond), the row sums, and eq. filter_mat on seeded inputs."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import filt
from synth import clouds, fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _edm(mid, rmin):
    from paper_2012_08208_amd import EdmFilter
    t = torch.as_tensor(mid, dtype=torch.float64, device="cuda:0")
    return EdmFilter(t, rmin)


def _csr(e):
    n = e.n
    rowptr = e.rowptr.cpu().numpy()
    col = e.col.cpu().numpy()[: e.nnz]
    w = e.w.cpu().numpy()[: e.nnz]
    return rowptr, col, w, sp.csr_matrix((w, col, rowptr), shape=(n, n))


def _check_csr(e, pts, rmin):
    rowptr, col, w, Wg = _csr(e)
    n = pts.shape[0]
    assert rowptr[0] == 0 and np.all(np.diff(rowptr) >= 1)    # the diagonal is always there
    for a in range(0, n, max(1, n // 257)):                     # no duplicate columns
        cols = col[rowptr[a]: rowptr[a + 1]]
        assert np.unique(cols).size == cols.size
    assert np.all(w > 0) and np.all(w <= rmin)
    Wo = filt.weights_sparse(pts, rmin)
    diff = abs(Wg - Wo)
    # pairs within rounding of the radius may appear on one side only, with
    # weights of that rounding's size
    assert (diff.max() if diff.nnz else 0.0) <= 4e-15 * rmin
    assert abs(Wg.nnz - Wo.nnz) <= max(2, Wo.nnz // 100000)
    R = e.R.cpu().numpy()[:n]
    Ro = filt.row_sums(Wo)
    assert np.max(np.abs(R - Ro) / Ro) <= 1e-13
    return Wo, Ro


CASES = [
    ("2d", (120, 60), 21, 1.5, 3, None),
    ("2d-neg", (64, 40), 22, 3.0, 2, (-5.0e5, -2.5e3)),
    ("3d", (24, 12, 12), 23, 2.5, 2, None),
    ("3d-shift", (18, 10, 9), 24, 1.6, 1, (-3.3, 1.0e6, -2.0e4)),
]


@pytest.mark.parametrize("name,nel,seed,rmin,holes,origin", CASES, ids=[c[0] for c in CASES])
def test_weights_rowsums_and_filter_match_oracle(name, nel, seed, rmin, holes, origin):
    mid = clouds.cloud(nel, seed, holes=holes, origin=origin)
    pts = mid.T
    n = pts.shape[0]
    print(f"edm case {name}: n={n} rmin={rmin}", flush=True)
    e = _edm(mid, rmin)
    Wo, Ro = _check_csr(e, pts, rmin)
    rho = fields.rho_random(seed + 1, n, lo=1e-3, hi=1.0)
    dc = -np.abs(fields.rho_random(seed + 2, n, lo=1e-6, hi=10.0))
    want = filt.apply(Wo, Ro, rho, dc)
    rt = torch.as_tensor(rho, device="cuda:0")
    dt = torch.as_tensor(dc, device="cuda:0")
    out = torch.empty_like(rt)
    e.filter(rt, dt, out)
    got = out.cpu().numpy()
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12
    out2 = torch.empty_like(rt)
    e.filter(rt, dt, out2)
    assert torch.equal(out, out2)                       # fixed-order reductions


def test_build_is_deterministic():
    mid = clouds.cloud((20, 10, 8), 31, holes=2)
    a, b = _edm(mid, 2.5), _edm(mid, 2.5)
    assert a.nnz == b.nnz
    for x, y in ((a.rowptr, b.rowptr), (a.col[: a.nnz], b.col[: b.nnz]), (a.w[: a.nnz], b.w[: b.nnz]),
                 (a.R, b.R)):
        assert torch.equal(x, y)


def test_degenerate_clouds():
    from paper_2012_08208_amd import EdmFilter
    # empty
    e = EdmFilter(torch.zeros((3, 0), dtype=torch.float64, device="cuda:0"), 1.0)
    assert e.nnz == 0 and int(e.rowptr[0]) == 0
    # one point: W = [[rmin]], s~ = s
    e = _edm(np.array([[0.25], [-3.0]]), 0.7)
    assert e.nnz == 1 and float(e.w[0]) == 0.7 and float(e.R[0]) == 0.7
    # radius below every spacing: W = rmin I, s~ = s exactly
    mid = clouds.cloud((30, 20), 41, jitter=0.0)
    e = _edm(mid, 0.2)
    n = mid.shape[1]
    assert e.nnz == n
    rho = torch.as_tensor(fields.rho_random(1, n, 0.1, 1.0), device="cuda:0")
    dc = torch.as_tensor(np.linspace(-3, -1, n), device="cuda:0")
    out = torch.empty_like(rho)
    e.filter(rho, dc, out)
    assert torch.allclose(out, dc, rtol=1e-15, atol=0)
    # all points in one place (one hash chunk holds everything)
    e = _edm(np.zeros((3, 300)), 1.0)
    assert e.nnz == 300 * 300
    assert torch.all(e.w[: e.nnz] == 1.0) and torch.all(e.R == 300.0)


def test_sampled_rows_at_a_large_cloud():
    """1.3M 3D midpoints (96x48x48 cubes, rmin 2.5, about 394 weights per
    row): sampled rows of the filter against the oracle's row-by-row form."""
    mid = clouds.cloud((96, 48, 48), 51, holes=3)
    pts = mid.T
    n = pts.shape[0]
    print(f"edm large: n={n}", flush=True)
    e = _edm(mid, 2.5)
    assert 300 * n < e.nnz < 450 * n
    rho = fields.rho_random(52, n, 1e-3, 1.0)
    dc = -np.abs(fields.rho_random(53, n, 1e-6, 1.0))
    rt, dt = torch.as_tensor(rho, device="cuda:0"), torch.as_tensor(dc, device="cuda:0")
    out = torch.empty_like(rt)
    e.filter(rt, dt, out)
    rows = np.random.default_rng(54).choice(n, 400, replace=False)
    want, Rw = filt.apply_rows(pts, 2.5, rho, dc, rows)
    got = out.cpu().numpy()[rows]
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12
    assert np.max(np.abs(e.R.cpu().numpy()[rows] - Rw) / Rw) <= 1e-13
