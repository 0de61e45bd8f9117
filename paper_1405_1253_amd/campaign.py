"""Long Rayleigh-Taylor runs and the mixing analysis of Sec. IV.

    python -m paper_1405_1253_amd.campaign --workload rt3_2400x6144_paper \\
        --tau-rt 4 --every 1000 --out run.npz

Every ``every`` steps the device computes the mixing objective (KE and
L_tot = L_u + L_d of eq. 3L) and, at a few chosen times, the row profiles of
T and E_k (Figs. 6, 8 and 9); only these small arrays come back to the host.
``alpha_tot`` turns the L_tot(t) series into the growth rate of eq. eqtot,
alpha_tot = Ldot_tot^2 / (4 At g L_tot) (the self-similar form of eq. eqL2).
"""
import argparse
import dataclasses
import json
import sys
import time

import numpy as np


def rt_time(wl, r):
    """RT time unit tau = sqrt(Lx / (g At)) (Sec. IV), Lx in length units."""
    return float(np.sqrt(r * wl.lx / (wl.g * wl.atwood)))


def alpha_tot(t, L, atwood, g):
    """Growth rate from the time series of the total mixing length:
    alpha = Ldot^2 / (4 At g L), Ldot by centred differences."""
    t = np.asarray(t, float)
    L = np.asarray(L, float)
    Ld = np.gradient(L, t)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(L > 0, Ld * Ld / (4.0 * atwood * g * L), np.nan)


def run(wl, nsteps, every, profile_times=(), progress=None, flags=0):
    import torch
    from . import abi
    from .runtime import Lattice
    lat = Lattice.from_workload(wl, flags=flags)
    t_rec, L_rec, Lu_rec, Ld_rec, ke_rec, prof = [], [], [], [], [], {}
    want = sorted(set(int(x) for x in profile_times))
    t = 0
    t0 = time.perf_counter()
    while True:
        if t % every == 0 or t in want:
            j = lat.objective().cpu().numpy()
            t_rec.append(t)
            ke_rec.append(j[1])
            L_rec.append(j[2])
            Lu_rec.append(j[3])
            Ld_rec.append(j[4])
            if not np.isfinite(j).all():
                raise FloatingPointError(f"state diverged at step {t}")
        if t in want:
            prof[t] = lat.profiles().cpu().numpy()
        if t >= nsteps:
            break
        n = min(every - t % every, nsteps - t)
        nxt = [w for w in want if w > t]
        if nxt:
            n = min(n, nxt[0] - t)
        lat.step(n)
        t += n
        if progress and t % (every * 10) == 0:
            progress(t, L_rec[-1], time.perf_counter() - t0)
    torch.cuda.synchronize()
    r = abi.lbm_lattice()[0]
    return {"t": np.array(t_rec), "L_tot": np.array(L_rec), "L_u": np.array(Lu_rec),
            "L_d": np.array(Ld_rec), "KE": np.array(ke_rec),
            "profile_steps": np.array(sorted(prof)),
            "profiles": np.array([prof[k] for k in sorted(prof)]),
            "tau_rt": rt_time(wl, r), "atwood": wl.atwood, "g": wl.g,
            "seconds": time.perf_counter() - t0}


def main(argv=None):
    from .workload import WORKLOADS
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--tau-rt", type=float, default=4.0, help="run length in RT time units")
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--profiles-at", type=str, default="0,1,2,3,4",
                    help="RT times at which to record the row profiles")
    ap.add_argument("--seed", type=int, default=None,
                    help="seed of the interface modes (default: the workload's); one realisation per seed")
    ap.add_argument("--precision", choices=("f64", "f32dev"), default=None,
                    help="population storage (default: the workload's; the paper's runs are double precision)")
    ap.add_argument("--collide-f64", action="store_true",
                    help="with f32dev storage: the collision in double arithmetic (LBM_COLLIDE_F64)")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    from . import abi
    wl = WORKLOADS[args.workload]
    if args.seed is not None:
        wl = dataclasses.replace(wl, seed=args.seed)
    if args.precision is not None:
        wl = dataclasses.replace(wl, precision=args.precision)
    tau = rt_time(wl, abi.lbm_lattice()[0])
    nsteps = int(round(args.tau_rt * tau / args.every)) * args.every
    ptimes = [int(round(float(x) * tau / args.every)) * args.every for x in args.profiles_at.split(",")]
    ptimes = [p for p in ptimes if p <= nsteps]
    print(json.dumps({"workload": wl.name, "seed": wl.seed, "precision": wl.precision,
                      "collide_f64": bool(args.collide_f64), "tau_rt_steps": tau, "nsteps": nsteps}), flush=True)

    def progress(t, L, s):
        print(f"step {t} (t/tau {t / tau:.2f}): L_tot {L:.1f}, {s:.0f} s", flush=True)

    out = run(wl, nsteps, args.every, ptimes, progress, flags=abi.COLLIDE_F64 if args.collide_f64 else 0)
    out["alpha_tot"] = alpha_tot(out["t"], out["L_tot"], out["atwood"], out["g"])
    np.savez(args.out, **out)
    print(json.dumps({"done": True, "seconds": out["seconds"], "steps": nsteps}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
