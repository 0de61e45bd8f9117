"""Runtime behaviour around the kernels: checkpoint/restore continues a run
bitwise, and a diverged state is reported (the divergence is forced from the
host by writing a NaN into the state; every kernel still runs normally)."""
import numpy as np
import pytest
import torch

from paper_1405_1253_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["rt3_128x384"])
@pytest.mark.parametrize("precision", ["f64", "f32dev"])
def test_checkpoint_restore_is_bitwise(tmp_path, name, precision):
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS[name]
    m = W.draw_modes(wl.seed)
    lat = Lattice(wl.lx, wl.lz, wl.tau, wl.g, precision=precision)
    lat.init_rt3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase, m.amp)
    lat.step(10)
    path = tmp_path / "ckpt.pt"
    lat.save(path)
    lat.step(15)
    straight = lat.state_soa().cpu().numpy()
    back = Lattice.load(path)
    assert back.steps_done == 10
    back.step(15)
    assert np.array_equal(back.state_soa().cpu().numpy(), straight)


def test_nonfinite_state_is_reported():
    from paper_1405_1253_amd.runtime import Lattice
    wl = W.WORKLOADS["rt3_128x384"]
    lat = Lattice.from_workload(wl)
    lat.step(3)
    lat.sums()                                   # finite: no error
    f = lat.state_soa()
    f[5, 17, 100] = float("nan")                 # forced from the host
    lat.set_state(f)
    lat.step(2)
    with pytest.raises(FloatingPointError):
        lat.sums()
    s = lat.sums(check=False).cpu().numpy()
    assert not np.isfinite(s).all()
