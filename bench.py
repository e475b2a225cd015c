"""Benchmark: MAC solves per second to a 1e-10 relative residual on one MI355X.

One step = one whole MAC projection as a time step of the method performs it
(Sec. 3.2 Steps 3/7): map the base state to face coefficients (fill + harmonic
faces + coefficient hierarchy), assemble the right-hand side, solve to
||r||/||b|| <= 1e-10, and correct the face velocity, on device-resident inputs
of the 256^3 plane-parallel workload (periodic x/y, Neumann z, 1e4 density
contrast, seeded).  `value` is the mixed-precision rate (FP32 V(2,2) cycles in
FP64 iterative refinement); the plain FP64 V-cycle rate is reported beside it.

The JSON line also carries the roofline of the dominant kernel (the finest-
level smoother, timed per launch with HIP events on the library's stream),
the FP64 CPU oracle timed on the host for a bounded sample, and the rate of
the nodal projection (Sec. 3.2 Step 11) on the same base state with a
cell-centred velocity (`nodal`, skipped with --no-nodal).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "MAC solves/sec to 1e-10 residual (mixed vs FP64) + stencil HBM GB/s"
WORKLOAD = "c2"


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=WORKLOAD, choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--fp64-steps", type=int, default=None, help="steps of the FP64 comparison (default: steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1, help="oracle projections timed on the host")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None, help="time one precision only")
    ap.add_argument("--no-nodal", action="store_true", help="skip the nodal-projection timing")
    ap.add_argument("--nodal-steps", type=int, default=10)
    ap.add_argument("--smoother", choices=["auto", "per_colour"], default="auto",
                    help="per_colour: one launch per colour on every level (the default runs both colours of a "
                         "finest-level sweep in one launch where rows are 128 or 256 cells)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB streaming copy (reference for the HBM traffic counters)")
    return ap.parse_args()


def _traffic_record(kernel):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    # the counters belong to the kernel source they were taken on
    import hashlib

    # (the .hip file and the headers it includes, hashed in the listed order)
    h = hashlib.sha256()
    for rel in rec.get("sources", []):
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        with open(src, "rb") as f:
            h.update(f.read())
    if not rec.get("sources") or h.hexdigest() != rec.get("sha256"):
        return None
    return rec


def _describe(p):
    bcs = "".join("PN"[b] for b in p.bc)
    if p.geometry == 0:
        shape = f"plane-parallel exponential atmosphere, {p.meta.get('contrast'):.0e} density contrast"
    else:
        shape = f"spherical star (linear radial fill at dr = h/5), {p.meta.get('contrast'):.0e} contrast to the box face"
    return f"{p.nx}x{p.ny}x{p.nz} {shape}, boundaries (x,y,z) {bcs}"


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solve is not sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1908_03634_amd import mproj, workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    dev = torch.device("cuda:0")
    p = W.config_problem(args.workload)
    n = p.ncell
    print(f"[bench] workload {p.name}: {p.nx}x{p.ny}x{p.nz}, bc {p.bc}", file=sys.stderr, flush=True)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    beta0_1d, rho, S = T(p.beta0_1d), T(p.rho), T(p.S)
    U0 = [T(p.ux), T(p.uy), T(p.uz)]
    K, Wm = args.steps, args.warmup

    def run(precision, steps, warmup):
        ctx = mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision=precision, rtol=1e-10,
                            smoother=args.smoother)
        total = steps + warmup
        # every step projects its own copy of the unprojected velocity
        copies = [[u.clone() for u in U0] for _ in range(total)]
        phi = ctx.empty_cells()
        infos = []
        torch.cuda.synchronize()
        t0 = None
        for s in range(total):
            if s == warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            # the last timed step also timestamps each finest-level smoother
            # launch (the roofline sample); the others run uninstrumented
            ctx.set_kernel_timing(s == total - 1)
            ctx.map_base_state(p.geometry, beta0_1d, rho, p.dr, p.center, want_coefs=False)
            _, info = ctx.mac_project(*copies[s], S, phi=phi)
            if s >= warmup:
                infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        del copies
        return dt, infos

    if args.copy_calibration:
        # a streaming kernel of known traffic (reads and writes 256 MiB each;
        # an elementwise product, so its name differs from every copy the
        # benchmark makes) to scale the HBM counters of the other kernels
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 elementwise copies reading and writing {nbytes} bytes each",
              file=sys.stderr, flush=True)
        del src, dst

    res = {}
    for prec in ("mixed", "fp64"):
        if args.only and prec != args.only:
            continue
        steps = K if prec == "mixed" else (args.fp64_steps or K)
        dt, infos = run(prec, steps, Wm)
        res[prec] = (dt, steps, infos)
        print(f"[bench] {prec}: {steps / dt:.2f} solves/s, {1e3 * dt / steps:.3f} ms/step, "
              f"steps {infos[-1]['outer_iters']}, rel {infos[-1]['rel_resid']:.2e}", file=sys.stderr, flush=True)

    main_prec = args.only or "mixed"
    dt, steps, infos = res[main_prec]
    value = steps / dt
    # dominant kernel: the finest-level red-black smoother (in mixed precision
    # on rows of 128 or 256 cells both colours of a sweep in one launch,
    # otherwise one launch per colour).  In the last timed step the library
    # timestamps each of its launches (HIP events recorded by the dispatch on
    # the library's stream) and adds up the algorithmic bytes of each launch:
    # x read (not from a zero start) and written, b and the cell coefficients
    # read, one word each per cell, plus 1/8 word of coarse correction after
    # prolongation and 16 bytes per cell where the refinement update rides on
    # the launch.
    tot_ms = sum(i["smooth_ms_total"] for i in infos)
    cnt = sum(i["smooth_launches"] for i in infos)
    tot_bytes = sum(i["smooth_bytes"] for i in infos)
    avg_s = tot_ms / cnt / 1e3 if cnt else float("nan")
    bytes_per_launch = tot_bytes / cnt if cnt else float("nan")
    achieved = bytes_per_launch / avg_s / 1e9
    if main_prec == "mixed":
        kname = "k_fsw_lds<float>" if infos[-1].get("smooth_form") == 1 else "k_gs_blk<float>"
    else:
        kname = "k_gs_blk<double>"
    rec = _traffic_record(f"{args.workload}:{kname}")
    traffic = None
    if rec:
        # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters,
        # averaged over the same launches as `achieved` and scaled by the
        # counters' reading of the calibration copy
        traffic = {"fetch_bytes": rec["fetch_bytes"], "write_bytes": rec["write_bytes"],
                   "total_bytes": rec["fetch_bytes"] + rec["write_bytes"],
                   "algorithmic_bytes": rec.get("algorithmic_bytes"), "calibration": rec.get("calibration"),
                   "summary": rec.get("summary")}
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic["total_bytes"] if traffic else None, "traffic_detail": traffic,
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": cnt,
                "bytes_per_launch": round(bytes_per_launch)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t0 = time.perf_counter()
        for _ in range(args.cpu_samples):
            r = oracle.mac_project(p, tol=1e-10)
        cdt = time.perf_counter() - t0
        cpu = {"value": round(args.cpu_samples / cdt, 4), "unit": "solves/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_samples} full {p.nx}x{p.ny}x{p.nz} projection(s) (fill, faces, rhs, FP64 "
                         f"V(2,2) multigrid to 1e-10 in {r['info']['cycles']} cycles, correction)"}
        print(f"[bench] cpu oracle: {cpu['value']} solves/s on {cpu['cores']} threads", file=sys.stderr, flush=True)

    last = infos[-1]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": Wm,
        "ms_per_step": round(1e3 * dt / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {_describe(p)}; map + rhs + solve to 1e-10 + "
                               f"velocity correction per step",
                   "precision": main_prec, "smoother": "red-black Gauss-Seidel V(2,2)",
                   "outer_steps": last["outer_iters"], "vcycles": last["vcycles"], "rel_resid": last["rel_resid"],
                   "levels": last["levels"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in res and main_prec != "fp64":
        fdt, fsteps, finfos = res["fp64"]
        line["fp64_value"] = round(fsteps / fdt, 3)
        line["fp64_ms_per_step"] = round(1e3 * fdt / fsteps, 4)
        line["fp64_cycles"] = finfos[-1]["vcycles"]
        line["mixed_over_fp64"] = round(value / (fsteps / fdt), 3)
    line["phase_ms"] = {"rhs": round(last["ms_rhs"], 4), "solve": round(last["ms_solve"], 4),
                        "correct": round(last["ms_correct"], 4)}
    if not args.no_nodal:
        line["nodal"] = _nodal(args, dev)
    print(json.dumps(line), flush=True)


def _nodal(args, dev):
    """The nodal projection of Sec. 3.2 Step 11 on the same base state with a
    cell-centred velocity: map + right-hand side + solve to 1e-10 + velocity
    correction per step, mixed precision."""
    import numpy as np
    import torch

    from paper_1908_03634_amd import mproj, workloads as W

    p = W.config_problem(args.workload, velocity="cells")

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    beta0_1d, rho, S = T(p.beta0_1d), T(p.rho), T(p.S)
    U0 = [T(p.ux), T(p.uy), T(p.uz)]
    ctx = mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision="mixed", rtol=1e-10)
    phi = ctx.empty_nodes()
    warm, steps = 2, args.nodal_steps
    U = [u.clone() for u in U0]
    info = None
    torch.cuda.synchronize()
    t0 = None
    for s in range(warm + steps):
        if s == warm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for u, u0 in zip(U, U0):
            u.copy_(u0)
        ctx.map_base_state(p.geometry, beta0_1d, rho, p.dr, p.center, want_coefs=False)
        _, info = ctx.nodal_project(*U, S, phi=phi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    out = {"workload": f"{args.workload} with cell-centred velocity: {_describe(p)}; nodes "
                       f"{'x'.join(str(m) for m in reversed(tuple(phi.shape)))}",
           "value": round(steps / dt, 3), "unit": "projections/s", "ms_per_step": round(1e3 * dt / steps, 4),
           "steps": steps, "precision": "mixed", "smoother": "4-colour Gauss-Seidel V(2,2)",
           "outer_steps": info["outer_iters"], "vcycles": info["vcycles"], "rel_resid": info["rel_resid"],
           "div_defect": round(info["div_defect"], 4),
           "phase_ms": {"rhs": round(info["ms_rhs"], 4), "solve": round(info["ms_solve"], 4),
                        "correct": round(info["ms_correct"], 4)},
           "note": "includes a device copy of the three unprojected velocity arrays per step"}
    print(f"[bench] nodal: {out['value']} projections/s, {out['ms_per_step']} ms/step", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
