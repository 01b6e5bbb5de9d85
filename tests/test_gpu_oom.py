"""DCDFT_ERR_OOM from dcdft_setup: a cell of 4096 fragments of 32^3 points with 80
orbitals each needs five FP64 orbital arrays of 86 GB, more than one GPU holds.
Setup must return the status (not crash), free what it allocated, and leave the
runtime usable: a small context set up afterwards runs a step and matches one set
up before (the failed allocation must not surface as an error of the next
context)."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu
from workloads.systems import RunConfig, Species, System
import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_setup_out_of_device_memory_then_a_normal_context():
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    from paper_2606_21125_amd.binding import DcdftError
    small = workloads.config(1)
    with DCDFT.from_config(small) as d0:
        e0 = d0.dcdft_scf_step()["e_total"]
    sp = Species("X", 2.0, -3.0, 1.0, 1.0, 1.0, 1.5)
    sysm = System(np.array([160.0, 160.0, 160.0]), np.array([[80.0, 80.0, 80.0]]),
                  np.zeros(1, dtype=np.int32), [sp])
    big = RunConfig("oom", sysm, (256, 256, 256), (16, 16, 16), (8, 8, 8),
                    np.full(4096, 80, dtype=np.int32), smearing=0.05)
    print("setting up the oversized cell", flush=True)
    with pytest.raises(DcdftError) as err:
        DCDFT.from_config(big)
    print("status:", err.value, flush=True)
    assert "DCDFT_ERR_OOM" in str(err.value)
    with DCDFT.from_config(small) as d1:
        e1 = d1.dcdft_scf_step()["e_total"]
    assert e1 == e0
