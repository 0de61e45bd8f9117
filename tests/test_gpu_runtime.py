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


@pytest.mark.parametrize("inplace,wall", [(False, "dirichlet"), (True, "diffuse")])
def test_tune_placement_keeps_the_run(inplace, wall):
    """Re-allocating the buffers for speed changes nothing of the run: the
    state after tuning is the state before it, bit for bit, and the steps
    after it give what an untuned lattice gives (also with an odd number of
    in-place steps done, i.e. the single buffer in its streamed form)."""
    from paper_1405_1253_amd.runtime import Lattice
    from paper_1405_1253_amd import abi
    wl = W.WORKLOADS["rt3_128x384"]
    m = W.draw_modes(wl.seed)
    flags = abi.wall_flag(wall)
    lats = []
    for _ in range(2):
        lat = Lattice(24, 1100, wl.tau, 1e-4, flags=flags, inplace=inplace)
        lat.init_rt3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase, m.amp)
        lat.step(3)
        lats.append(lat)
    raw = lats[0].buf[lats[0].cur].clone()
    times = lats[0].tune_placement(trials=3, steps=4)
    assert times is not None and len(times) == 3 and all(t > 0 for t in times)
    assert lats[0].steps_done == 3
    assert torch.equal(lats[0].buf[lats[0].cur].view(torch.uint8), raw.view(torch.uint8))
    for lat in lats:
        lat.step(5)
    a, b = (l.state_soa().cpu().numpy() for l in lats)
    assert np.array_equal(a, b)
