"""The ps2 split's SVD (tenso_svd_truncate) on synthetic two-site tensors
with prescribed spectra from 1 down to 1e-12, against numpy's SVD (LAPACK)
and the oracle's truncation rule.

Theta = U diag(s) V^H with Haar-random unitaries; the cases cover the shapes
of the structured-bath ternary tree at rank cap 8 (up to 512 x 1000), a side
above the blocked QR's 1024 rows, a side below the 64 test columns (exact
factorisation), an exactly rank-deficient tensor, and a numerical rank above
64 (power steps).  Bars: singular values within 1e-13 s_1 (the leading 32
when the numerical rank exceeds the 64 captured directions); the kept
subspace (leading singular directions whose gap to the next value is at
least 1e-6 s_1) within 1e-9 of LAPACK's; the decision (r', k, r_eps) equal to
the oracle's for eps in {1e-10, 1e-8, 1e-6, 1e-3} and caps {8, 64}, and with
eps = 0 every direction kept up to the cap."""
import numpy as np
import pytest

from oracle.integrators import SVD_ZERO_TOL, Propagator
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def haar(n, k, rng):
    z = rng.normal(size=(n, k)) + 1j * rng.normal(size=(n, k))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def make(rows, cols, s, rng):
    k = len(s)
    return (haar(rows, k, rng) * s) @ haar(cols, k, rng).conj().T


CASES = [
    ("512x1000 geometric 40", 512, 1000, np.logspace(0, -12, 40)),
    ("1000x210 geometric 30", 1000, 210, np.logspace(0, -12, 30)),
    ("300x500 geometric 50", 300, 500, np.logspace(0, -12, 50)),
    ("2000x100 geometric 60 (QR above 1024 rows)", 2000, 100, np.logspace(0, -12, 60)),
    ("40x700 exact (p = smaller side)", 40, 700, np.logspace(0, -12, 40)),
    ("256x256 rank 5", 256, 256, np.array([1.0, 0.3, 1e-3, 1e-7, 1e-11])),
    ("600x800 rank 90 (power steps)", 600, 800, np.logspace(0, -12, 90)),
    ("64x4096 plateau", 64, 4096, np.r_[np.ones(4), np.logspace(-2, -12, 30)]),
]


@pytest.mark.parametrize("name,rows,cols,spec", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("iso", [0, 1])
def test_svd_truncate_matches_lapack(name, rows, cols, spec, iso):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[svd] {name}, iso {iso}", flush=True)
    rng = np.random.default_rng(rows * 7 + cols + iso)
    A = make(rows, cols, spec, rng)
    U, S, Vh = np.linalg.svd(A, full_matrices=False)
    p = min(64, rows, cols)
    sig, vec, dec, missed = api.svd_truncate(A, iso=iso, eps=1e-6, max_rank=64)
    assert len(sig) == p
    nc = p if len(spec) <= p else 32
    err_s = np.abs(sig[:nc] - S[:nc]).max() / S[0]
    ref = U[:, :p] if iso == 0 else Vh[:p].conj().T
    # subspaces of the leading j directions, for every j with a clear gap
    worst = 0.0
    for j in range(1, min(nc, len(spec))):
        if S[j - 1] - S[j] < 1e-6 * S[0]:
            continue
        Pg = vec[:, :j] @ vec[:, :j].conj().T
        Pn = ref[:, :j] @ ref[:, :j].conj().T
        worst = max(worst, np.abs(Pg - Pn).max())
    print(f"  max |s - s_lapack| / s_1 = {err_s:.2e}; subspace error {worst:.2e}; "
          f"missed energy {missed:.1e}; decision {dec}", flush=True)
    assert err_s < 1e-13
    assert worst < 1e-9
    r_eps_o = None
    for eps in (1e-10, 1e-8, 1e-6, 1e-3):
        for cap in (8, 64):
            _, _, d, _ = api.svd_truncate(A, iso=iso, eps=eps, max_rank=cap)
            rp = Propagator.truncation_rank(S, eps, cap, min(rows, cols))
            k = min(int(np.sum(S > SVD_ZERO_TOL * S[0])), rp)
            assert (d[0], d[1]) == (rp, k), (eps, cap, d, rp, k)
            if eps == 1e-6:
                # r_eps is exact when it lies within the p computed directions
                # (p = 2 cap + 8 for cap 8), else reported as min(rows, cols)
                p_used = min(64, rows, cols, 2 * min(cap, rows, cols) + 8)
                r_eps_o = Propagator.truncation_rank(S, eps, 10 ** 6, 10 ** 6, grow=0)
                want = r_eps_o if r_eps_o < p_used else min(rows, cols)
                assert d[2] == want, (d, r_eps_o, p_used)
    for cap in (8, 64):
        _, _, d, _ = api.svd_truncate(A, iso=iso, eps=0.0, max_rank=cap)
        assert d[0] == min(cap, rows, cols), (cap, d)


def test_svd_truncate_errors():
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    with pytest.raises(TensoError) as e:
        api.svd_truncate(np.zeros((4, 4)), iso=2)
    assert e.value.code == "EINVAL"
    with pytest.raises(TensoError) as e:
        api.svd_truncate(torch.zeros((1 << 14, 1 << 13), dtype=torch.complex128, device="cuda"))
    assert e.value.code == "ENOMEM"


def test_svd_truncate_narrow_width_for_a_small_cap():
    """With max_rank 8 the factorisation uses 24 test columns (2 * 8 + 8) and
    power steps: the leading 9 singular values and the kept subspace still
    match LAPACK, and the decision equals the oracle's."""
    require_gpu()
    from paper_2603_17711_amd import api
    rng = np.random.default_rng(5)
    for rows, cols, spec in [(512, 1000, np.logspace(0, -12, 40)),
                             (1000, 210, np.logspace(0, -6, 60))]:
        A = make(rows, cols, spec, rng)
        U, S, Vh = np.linalg.svd(A, full_matrices=False)
        sig, vec, dec, missed = api.svd_truncate(A, iso=0, eps=1e-6, max_rank=8)
        assert len(sig) == 24
        err_s = np.abs(sig[:9] - S[:9]).max() / S[0]
        Pg = vec[:, :8] @ vec[:, :8].conj().T
        Pn = U[:, :8] @ U[:, :8].conj().T
        rp = Propagator.truncation_rank(S, 1e-6, 8, min(rows, cols))
        k = min(int(np.sum(S > SVD_ZERO_TOL * S[0])), rp)
        print(f"[svd] {rows}x{cols} cap 8: s error {err_s:.1e}, subspace "
              f"{np.abs(Pg - Pn).max():.1e}, decision {dec} vs oracle ({rp}, {k})")
        assert err_s < 1e-13 and np.abs(Pg - Pn).max() < 1e-9
        assert (dec[0], dec[1]) == (rp, k)
