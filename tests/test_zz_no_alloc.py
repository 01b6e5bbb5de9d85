"""dcdft_band_energy_noalloc (static device scratch, no allocation) against
dcdft_band_energy (the context's scratch), through the C ABI, on two calls in a
row on the same GPU, the second with a smaller input.

Both compute H psi per vector with the same kernels, so H psi-derived outputs
(grad_psi) and grad_v agree bit for bit; the energy is summed over chunks of
different sizes (the static array holds a different number of vectors than the
context's m_pad chunk), so it agrees to FP64 rounding (relative 1e-13).  The
first call uses more vectors than either chunk, so both paths cut it into chunks.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu
import workloads

pytestmark = pytest.mark.gpu


def _run(d, fn_name, frag, x, f, veff, prec):
    import torch
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    gp = torch.empty_like(x)
    gv = torch.empty(veff.numel(), dtype=torch.float64, device="cuda")
    getattr(d, fn_name)(frag, x, f, veff=veff, energy=e, grad_psi=gp, grad_v=gv, prec=prec)
    torch.cuda.synchronize()
    return float(e), gp.cpu().numpy(), gv.cpu().numpy()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_matches_band_energy_on_two_calls(dtype):
    require_gpu()
    import torch
    from paper_2606_21125_amd import DCDFT
    cfg = workloads.config(1)           # 8 fragments of 24^3 points, 64 orbitals
    prec = 0 if dtype == "float64" else 1
    tdt = getattr(torch, dtype)
    rng = np.random.default_rng(77)
    with DCDFT.from_config(cfg, precision=prec) as d:
        d.dcdft_scf_step()
        n = d.n
        for frag, m in ((3, 150), (6, 5)):
            print("noalloc call: fragment", frag, "vectors", m, dtype, flush=True)
            x = torch.tensor(rng.normal(size=(m, n)), device="cuda", dtype=tdt)
            f = torch.tensor(rng.uniform(0.0, 2.0, size=m), device="cuda")
            veff = torch.tensor(rng.normal(size=n), device="cuda")
            ea, gpa, gva = _run(d, "dcdft_band_energy", frag, x, f, veff, prec)
            eb, gpb, gvb = _run(d, "dcdft_band_energy_noalloc", frag, x, f, veff, prec)
            assert np.array_equal(gpa, gpb)
            assert np.array_equal(gva, gvb)
            assert abs(ea - eb) <= 1e-13 * max(1.0, abs(ea)), (ea, eb)
