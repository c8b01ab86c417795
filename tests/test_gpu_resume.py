"""Checkpoint and resume: export the state at step 100 (FP64, canonical
order), import it into a fresh context, run 100 more steps, and require the
result to equal an uninterrupted 200-step run bit for bit.  This holds for
every storage kind because the export is exact (FP64 and FP32 values, and
shifted 16-bit values w_a rho_ref + h, survive FP64 and back) and the step's
arithmetic depends only on the state and, for the stochastically rounded
f16m/bf16m, on the step number, which the checkpoint carries."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STORAGES = ["f64", "f32", "f16s", "bf16s", "f16m", "bf16m"]


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_11792_amd import lbm as mod

    return mod


@pytest.mark.parametrize("storage", STORAGES)
def test_resume_is_bitwise(lbm, storage):
    nx, ny, nz, tau, G = 40, 36, 64, 0.85, -5.5
    spec = dict(R0=8.0, amp_rel=0.1, wavelength=32.0, rho_l=2.29, rho_v=0.087, noise_amp=1e-3, seed=9)
    full = lbm.Lattice(nx, ny, nz, tau, G, storage=storage, rho_ref=0.087)
    full.init_ligament(**spec)
    full.step(100)
    checkpoint = full.populations().cpu().numpy()
    full.step(100)
    ref = full.populations().cpu().numpy()
    full.close()

    resumed = lbm.Lattice(nx, ny, nz, tau, G, storage=storage, rho_ref=0.087)
    resumed.set_populations(checkpoint)
    resumed.set_step(100)  # the stochastic rounding of f16m/bf16m is keyed by the step
    assert np.array_equal(resumed.populations().cpu().numpy(), checkpoint)
    resumed.step(100)
    got = resumed.populations().cpu().numpy()
    assert np.array_equal(got, ref)
    resumed.close()
