"""Droplet labelling on the device (lbm_droplets) against the oracle's flood
fill: the 6-connected periodic components of rho > rho_mid.

Random two-valued density fields (liquid 2.0 with probability p, vapour 0.1
otherwise) are imported as rest populations, so the mask is known exactly;
p spans the site-percolation threshold of the cubic lattice (about 0.3116),
where cluster sizes spread over all scales and components wrap around the
periodic faces.  Counts, (volume, first node) pairs and the order are
compared exactly, masses to 1e-12.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
MID = 1.05


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_11792_amd import lbm as mod

    return mod


def _expected(oracle_mod, rho):
    """(count, [(volume, first_node, mass)] sorted by volume desc, first node asc)."""
    count, lab = oracle_mod.label(rho, MID)
    flat = lab.ravel()
    r = rho.ravel()
    out = []
    for k in range(1, count + 1):
        idx = np.nonzero(flat == k)[0]
        out.append((idx.size, int(idx[0]), float(r[idx].sum())))
    out.sort(key=lambda t: (-t[0], t[1]))
    return count, out


def _device(lbm, rho, storage="f64"):
    import torch

    nz, ny, nx = rho.shape
    lat = lbm.Lattice(nx, ny, nz, 0.8, -5.5, storage=storage, rho_ref=0.1)
    pop = torch.tensor(W[:, None, None, None] * rho[None], dtype=torch.float64, device="cuda")
    lat.set_populations(pop)
    d = lat.droplets(MID, max_out=1 << 20)
    lat.close()
    return d


def _compare(d, exp):
    count, items = exp
    assert d["count"] == count
    got = list(zip(d["volumes"].tolist(), d["first_nodes"].tolist()))
    assert got == [(v, f) for v, f, _ in items]
    assert np.allclose(d["masses"], [m for _, _, m in items], rtol=1e-12, atol=0)


@pytest.mark.parametrize("shape,p,seed", [
    ((29, 23, 17), 0.2, 1), ((29, 23, 17), 0.3116, 2), ((29, 23, 17), 0.5, 3),
    ((40, 48, 64), 0.3116, 4), ((40, 1, 1), 0.5, 5), ((5, 3, 2), 0.5, 6), ((7, 1, 5), 0.6, 7),
    ((1, 1, 1), 1.0, 8), ((2, 1, 2), 0.5, 9),
])
def test_random_masks_match_oracle(lbm, oracle_mod, shape, p, seed):
    rng = np.random.default_rng(seed)
    rho = np.where(rng.random(shape) < p, 2.0, 0.1)
    _compare(_device(lbm, rho), _expected(oracle_mod, rho))


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_other_storage_kinds(lbm, oracle_mod, storage):
    rng = np.random.default_rng(11)
    rho = np.where(rng.random((24, 20, 18)) < 0.3116, 2.0, 0.1)
    d = _device(lbm, rho, storage)
    count, items = _expected(oracle_mod, rho)
    assert d["count"] == count
    assert list(zip(d["volumes"].tolist(), d["first_nodes"].tolist())) == [(v, f) for v, f, _ in items]
    tol = 1e-6 if storage == "f32" else 2e-3
    assert np.allclose(d["masses"], [m for _, _, m in items], rtol=tol)


def test_degenerate_fields(lbm):
    shape = (8, 4, 6)
    n = 8 * 4 * 6
    d = _device(lbm, np.full(shape, 0.1))
    assert d["count"] == 0 and d["volumes"].size == 0
    d = _device(lbm, np.full(shape, 2.0))
    assert d["count"] == 1 and d["volumes"].tolist() == [n] and d["first_nodes"].tolist() == [0]
    assert d["masses"][0] == pytest.approx(2.0 * n, rel=1e-14)
    # checkerboard: no two liquid nodes share a face, also across the periodic faces
    z, y, x = np.indices(shape)
    rho = np.where((x + y + z) % 2 == 0, 2.0, 0.1)
    d = _device(lbm, rho)
    assert d["count"] == n // 2
    assert (d["volumes"] == 1).all()
    assert d["first_nodes"].tolist() == sorted(np.nonzero(rho.ravel() > MID)[0].tolist())
    # non-finite densities are background
    rho = np.full(shape, 2.0)
    rho[:, :, 3] = np.nan
    d = _device(lbm, rho)
    assert d["count"] == 1 and d["volumes"].tolist() == [n - 8 * 4]


def test_max_out_and_order(lbm, oracle_mod):
    rng = np.random.default_rng(21)
    rho = np.where(rng.random((16, 16, 16)) < 0.25, 2.0, 0.1)
    count, items = _expected(oracle_mod, rho)
    import torch

    lat = lbm.Lattice(16, 16, 16, 0.8, -5.5, storage="f64")
    lat.set_populations(torch.tensor(W[:, None, None, None] * rho[None], device="cuda"))
    d = lat.droplets(MID, max_out=3)
    assert d["count"] == count and d["volumes"].tolist() == [v for v, _, _ in items[:3]]
    d0 = lat.droplets(MID, max_out=0)
    assert d0["count"] == count and d0["volumes"].size == 0
    lat.close()


def test_labelling_leaves_the_state_untouched(lbm):
    s = workloads.SMALL_FP64
    kw = dict(R0=s.R0, amp_rel=s.amp_rel, wavelength=s.wavelength, rho_l=2.3068, rho_v=0.1041)
    a = lbm.Lattice(s.nx, s.ny, s.nz, s.tau, s.G, storage="f32")
    b = lbm.Lattice(s.nx, s.ny, s.nz, s.tau, s.G, storage="f32")
    a.init_ligament(**kw)
    b.init_ligament(**kw)
    a.step(31)
    b.step(31)
    assert a.droplets(MID)["count"] == 1
    a.step(31)
    b.step(31)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.close()
    b.close()


def test_after_breakup_matches_host_labelling(lbm):
    from paper_1904_11792_amd import analysis

    s = workloads.SMALL_FP64
    lat = lbm.Lattice(s.nx, s.ny, s.nz, s.tau, s.G, storage="f64")
    rl, rv = 2.306807, 0.104100
    lat.init_ligament(R0=s.R0, amp_rel=s.amp_rel, wavelength=s.wavelength, rho_l=rl, rho_v=rv)
    lat.step(1200)
    mid = 0.5 * (rl + rv)
    host = analysis.droplets(lat.fields()["rho"].cpu().numpy(), mid)
    dev = lat.droplets(mid)
    lat.close()
    assert dev["count"] == host.count >= 1
    assert dev["volumes"].tolist() == host.volumes.tolist()
    assert np.allclose(dev["masses"], host.masses, rtol=1e-12)
