"""FP32 deviation storage against FP64 on the same workload.

    python -m paper_1405_1253_amd.precision fields   [--steps 20000] [--collide-f64]
    python -m paper_1405_1253_amd.precision gradient [--steps 5000] [--collide-f64]
    python -m paper_1405_1253_amd.precision interface [--steps 20000]

fields:   the 4096 x 12288 three-layer workload is run in FP64 and in FP32
          deviation storage for the same number of steps; the renormalised
          fields (rho, u^H_x, u^H_z, T^H) are compared site by site (max and
          RMS absolute error per field, and the max relative error of rho and
          T) and the mixing lengths of both fronts (L_u, L_d, their sum) and
          KE of both runs are printed.
gradient: dJ/d amp of the 2048 x 6144 rollout with FP32 storage and float
          adjoint buffers against the same rollout in FP64 throughout.
interface: the double-front workload of the paper's runs (Sec. IV, 6144
          rows, 64 columns) with flat interfaces (zero amplitudes: the
          fronts only diffuse, every column alike) at tau = 0.50546 (the
          paper's), 0.52 and 0.7: L_u + L_d in FP32 deviation storage (float
          collision, and double collision with LBM_COLLIDE_F64) over FP64
          after 2,000 steps and after the given number.
Each mode prints one JSON line.  All arithmetic runs in the library's kernels;
differences are reduced on the device with torch.
"""
import argparse
import json
import sys
import time

import torch


def _field_errors(a, b):
    names = ("rho", "u_x", "u_z", "T")
    out = {}
    for i, n in enumerate(names):
        d = (a[i] - b[i]).abs()
        out[n] = {"max_abs": float(d.max()), "rms": float(d.pow(2).mean().sqrt())}
        if n in ("rho", "T"):
            out[n]["max_rel"] = float((d / b[i].abs()).max())
    return out


def fields(steps, collide_f64=False):
    from . import abi
    from .runtime import Lattice
    from .workload import WORKLOADS
    res = {"mode": "fields", "steps": steps, "collide_f64": collide_f64}
    t0 = time.perf_counter()
    lat64 = Lattice.from_workload(WORKLOADS["rt3_4096x12288"])
    lat32 = Lattice.from_workload(WORKLOADS["rt3_4096x12288_f32"], flags=abi.COLLIDE_F64 if collide_f64 else 0)
    done = 0
    while done < steps:
        n = min(2000, steps - done)
        lat64.step(n)
        lat32.step(n)
        done += n
        torch.cuda.synchronize()
        print(f"step {done}: {time.perf_counter() - t0:.0f} s", flush=True)
    lat64.sums()
    lat32.sums()
    f64 = lat64.fields()
    f32 = lat32.fields()
    res["errors"] = _field_errors(f32, f64)
    j64 = lat64.objective().cpu().tolist()
    j32 = lat32.objective().cpu().tolist()
    res["mixing_length_f64"], res["mixing_length_f32"] = j64[2], j32[2]
    res["L_u_f64"], res["L_u_f32"] = j64[3], j32[3]
    res["L_d_f64"], res["L_d_f32"] = j64[4], j32[4]
    res["ke_f64"], res["ke_f32"] = j64[1], j32[1]
    res["seconds"] = time.perf_counter() - t0
    return res


def gradient(steps, collide_f64=False):
    from .rollout import Rollout, RolloutConfig
    from .workload import WORKLOADS, draw_modes
    wl = WORKLOADS["rt3_2048x6144_adj"]
    m = draw_modes(wl.seed)
    amp = torch.as_tensor(m.amp, device="cuda")
    grads = {}
    t0 = time.perf_counter()
    for prec, adj in (("f32dev", "f32"), ("f64", "f64")):
        r = Rollout(RolloutConfig.from_workload(wl, m, nsteps=steps, precision=prec, adj_precision=adj,
                                                mom_precision=adj, moment_budget_bytes=40 << 30,
                                                collide_f64=collide_f64 and prec == "f32dev"))
        J = r.forward(amp)[0].item()
        grads[prec] = (J, r.backward())
        del r
        torch.cuda.empty_cache()
        print(f"{prec} rollout done: {time.perf_counter() - t0:.0f} s", flush=True)
    (J32, g32), (J64, g64) = grads["f32dev"], grads["f64"]
    err = (g32 - g64).abs()
    return {"mode": "gradient", "steps": steps, "collide_f64": collide_f64, "J_f64": J64, "J_f32": J32,
            "J_rel_err": abs(J32 / J64 - 1), "grad_max_abs_err": float(err.max()),
            "grad_max_err_over_max_grad": float(err.max() / g64.abs().max()),
            "grad_rms_rel_err": float((err.pow(2).mean() / g64.pow(2).mean()).sqrt()),
            "seconds": time.perf_counter() - t0}


def interface(steps):
    import dataclasses
    import numpy as np
    from .runtime import Lattice
    from .workload import WORKLOADS, draw_modes
    base = WORKLOADS["rt3_2400x6144_paper"]
    m = draw_modes(base.seed)
    res = {"mode": "interface", "workload": base.name, "lx": 64, "steps": [0, 2000, steps], "L_tot": {}}
    t0 = time.perf_counter()
    from . import abi
    for tau in (base.tau, 0.52, 0.7):
        row = {}
        for key, prec, flags in (("f64", "f64", 0), ("f32dev", "f32dev", 0),
                                 ("f32dev_collide_f64", "f32dev", abi.COLLIDE_F64)):
            lat = Lattice.from_workload(dataclasses.replace(base, lx=64, tau=tau, precision=prec), modes=m,
                                        amp=np.zeros_like(m.amp), flags=flags)
            vals, done = [float(lat.objective()[2])], 0
            for n in (2000, steps):
                lat.step(n - done)
                done = n
                vals.append(float(lat.objective()[2]))
            row[key] = vals
        row["f32_over_f64"] = [b / a for a, b in zip(row["f64"], row["f32dev"])]
        row["f32_collide_f64_over_f64"] = [b / a for a, b in zip(row["f64"], row["f32dev_collide_f64"])]
        res["L_tot"][f"tau={tau}"] = row
    res["seconds"] = time.perf_counter() - t0
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("fields", "gradient", "interface"))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--collide-f64", action="store_true", help="fields, gradient: the FP32 run collides in double")
    a = ap.parse_args(argv)
    if a.mode == "fields":
        out = fields(a.steps or 20000, a.collide_f64)
    elif a.mode == "interface":
        out = interface(a.steps or 20000)
    else:
        out = gradient(a.steps or 5000, a.collide_f64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
