"""Long-run parity on the small FP64 ligament (32 x 32 x 64, tau 1, G -5.5,
R0 = 6 (1 + 0.1 cos(2 pi z / 64))): run through pinch-off to step 2000 on the
GPU and in the oracle.  Bars: break-up time within 1%, the same droplet
count with volumes within 1%, and the same total mass."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

STEPS = 2000


@pytest.fixture(scope="module")
def oracle_run(oracle_mod):
    s = workloads.SMALL_FP64
    co = oracle_mod.coexistence(s.G, s.tau)
    f0 = oracle_mod.init_ligament(s.nx, s.ny, s.nz, R0=s.R0, amp_rel=s.amp_rel,
                                  wavelength=s.wavelength, rho_l=co.rho_l, rho_v=co.rho_v)
    mid = 0.5 * (co.rho_l + co.rho_v)
    tb, steps, necks, f = oracle_mod.run_to_breakup(f0, s.tau, s.G, mid, STEPS)
    f = oracle_mod.run(f, STEPS - steps[-1], s.tau, s.G)
    rho = f.sum(axis=0)
    count, vols, mass = oracle_mod.droplets(rho, mid)
    return {"co": co, "tb": tb, "count": count, "vols": vols, "mass_total": oracle_mod.diag(f)["mass"],
            "m0": oracle_mod.diag(f0)["mass"]}


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_small_ligament_breakup_parity(oracle_mod, oracle_run, storage):
    import torch

    from paper_1904_11792_amd import analysis, lbm

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = workloads.SMALL_FP64
    co = oracle_run["co"]
    lat = lbm.Lattice(s.nx, s.ny, s.nz, s.tau, s.G, storage=storage)
    lat.init_ligament(R0=s.R0, amp_rel=s.amp_rel, wavelength=s.wavelength, rho_l=co.rho_l, rho_v=co.rho_v)
    tb, steps, necks, last = analysis.run_to_breakup(lat, co.rho_l, co.rho_v, STEPS, every=1)
    assert oracle_run["tb"] is not None and tb is not None
    print(f"{storage}: break-up at {tb:.2f} steps (oracle {oracle_run['tb']:.2f})")
    assert tb == pytest.approx(oracle_run["tb"], rel=0.01)
    lat.step(STEPS - lat.step_count)
    mid = 0.5 * (co.rho_l + co.rho_v)
    d = analysis.droplets(lat.fields()["rho"].cpu().numpy(), mid)
    assert d.count == oracle_run["count"]
    assert np.allclose(d.volumes, oracle_run["vols"], rtol=0.01)
    mass = lat.diagnostics()["mass"]
    tol = 1e-12 if storage == "f64" else 1e-5
    assert mass == pytest.approx(oracle_run["mass_total"], rel=tol)
    assert mass == pytest.approx(oracle_run["m0"], rel=tol)
