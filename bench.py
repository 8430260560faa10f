"""Benchmark: flux-reconstruction Navier-Stokes RHS with flux anti-aliasing.

One step = one full right-hand-side evaluation (all kernel groups) of the
Taylor-Green vortex state on a 48^3 periodic hexahedral mesh, p = 3, with
6^3 Gauss-Legendre anti-aliasing points per element, fused kernels with
FP32 bulk arithmetic and FP64 state.  value = whole-job GDoF-RHS/s, with
DoF = 5 conserved variables x solution points (7.08M points, 35.4M DoF).
The same run reports the FP64 fused path and p = 4 alongside, the volume
kernel's HBM/ALU roofline position measured with HIP events, and the
reference oracle timed on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF-RHS/s NS+AA FR (fused FP32 vs plain FP64), % HBM roofline; p99 step ms"
HBM_PEAK_GBS = 8000.0
# vector ALU peak from unit counts: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz.
# FP64 FMA runs at full rate; FP32 reaches twice this only with packed math,
# which this build does not emit.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# HBM bytes per launch of hex_volume<3, float> on the 48^3 workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from
# a 1 GiB copy), profiles/hex_fused_fp32_p3_tgv48.md.  Valid for the kernel as
# profiled; None once the kernel changes.
HEX_VOL_P3_FP32_TRAFFIC = (270601.6 * 2 + 304128.0) * 1024


def volume_model(p, bytes_real):
    """Algorithmic HBM bytes and FLOPs of one element in the fused volume
    kernel (hex).  Bytes: state read (5 N_u doubles), neighbour face states
    (5 N_f reals), normal viscous flux written (4 N_f reals), volume residual
    written (5 N_u reals), face records + per-element metrics (small).
    FLOPs: the sum-factorised sweeps, gradient, the point-wise flux at the
    m^3 quadrature points (about 130 flops each) and the face viscous fluxes."""
    n, m = p + 1, p + 3
    nu, nf = n ** 3, 6 * n * n
    byts = 5 * nu * 8 + 5 * nf * bytes_real + 4 * nf * bytes_real + 5 * nu * bytes_real + 6 * 8 + 10 * bytes_real
    fl = 0
    fl += 2 * 5 * 3 * n * n * n * 2                      # own face values (lb, rb)
    fl += 2 * 15 * nu * (n + 2)                           # corrected gradient
    fl += 2 * 15 * nu * 3                                 # J^-T
    fl += 2 * 20 * 3 * n * n * n * 2 + 3 * n * n * 2 * 60  # face interpolation + viscous normal flux
    fl += 2 * 20 * m * n * n * n                          # x sweep
    fl += 2 * 20 * m * m * n * n                          # y interpolation per column
    fl += 2 * 20 * m * m * m * n                          # z interpolation on the fly
    fl += m ** 3 * (130 + 2 * 45)                          # point flux + transformed flux
    fl += 2 * 15 * m ** 3 * n                             # z projection
    fl += 2 * 5 * m * n * (m * 3) * n                     # y projection
    fl += 2 * 5 * n * n * (2 * m) * n                     # x projection
    return byts, fl


def rhs_bytes_model(p, bytes_real):
    """Algorithmic bytes of one full fused RHS per element (hex): disu reads
    U and writes U^f; the volume group reads U and the neighbour U^f and
    writes V^f and the volume residual; the interface group reads the
    residual, own and neighbour U^f and V^f, and writes du."""
    n = p + 1
    nu, nf = n ** 3, 6 * n * n
    b = 5 * nu * 8 + 5 * nf * bytes_real
    b += 5 * nu * 8 + 5 * nf * bytes_real + 4 * nf * bytes_real + 5 * nu * bytes_real
    b += 5 * nu * bytes_real + 2 * 5 * nf * bytes_real + 2 * 4 * nf * bytes_real + 5 * nu * 8
    return b


def time_variant(frmi, torch, n, p, prec, steps, warmup, form="fused", kind="hex", aa=True, surface_aa=False):
    from paper_2401_06132_amd import inputs
    if form in ("noaa", "fullaa"):
        # the fused path without flux anti-aliasing (the paper's "AA off"), or
        # with flux and surface-flux anti-aliasing (its "full AA")
        aa, surface_aa, form = form == "fullaa", form == "fullaa", "fused"
    s = frmi.Solver(n, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0, form=form, aa=aa, surface_aa=surface_aa)
    coords = s.upts_coords()
    U = inputs.element_state(coords, seed=0)
    u = torch.from_numpy(np.concatenate([x.reshape(-1) for x in U])).cuda()
    del U, coords
    du = torch.empty_like(u)
    for _ in range(warmup):
        s.rhs(u, du)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        s.rhs(u, du)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    # dominant kernel (volume group) alone, same launch configuration
    vol_ms = float("nan")
    if form == "fused":
        for _ in range(max(1, warmup // 2)):
            s.rhs_stages(u, du, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            s.rhs_stages(u, du, 2)
        e1.record()
        torch.cuda.synchronize()
        vol_ms = e0.elapsed_time(e1) / steps
    ok = bool(torch.isfinite(du).all().item())
    res = dict(n_dof=s.n_state, n_elem=s.n_hex + s.n_prism + s.n_tet + s.n_pyr, wall_s=wall, ms_per_step=wall * 1e3 / steps,
               p50_ms=float(np.percentile(per, 50)), p99_ms=float(np.percentile(per, 99)), vol_ms=vol_ms,
               finite=ok)
    del s, u, du
    torch.cuda.empty_cache()
    return res


def run_rk(frmi, torch, kind, n, p, prec, nsteps, dt):
    """nsteps RK4 steps on the internal state; per-step HIP-event times and
    the drift of the conserved integrals."""
    from paper_2401_06132_amd import inputs
    s = frmi.Solver(n, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    U = inputs.element_state(s.upts_coords(), seed=0)
    s.set_state(np.concatenate([x.reshape(-1) for x in U]))
    del U
    c0 = s.integrals()
    s.rk4(dt, 1)  # warm-up step (not timed), part of the trajectory
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nsteps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(nsteps):
        s.rk4(dt, 1)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(nsteps)])
    c1 = s.integrals()
    st = s.get_state()
    finite = bool(np.isfinite(st).all())
    vol = (2 * np.pi) ** 3
    # drift relative to the integral itself (mass, energy) or to the mass
    # integral (momentum, whose integral is ~0 for the vortex)
    scale = np.array([abs(c0[0]), abs(c0[0]), abs(c0[0]), abs(c0[0]), abs(c0[4])])
    out = dict(workload="Taylor-Green vortex, %d^3-cell periodic box, %s, p=%d, %s, %d RK4 steps of dt=%g"
               % (n, kind, p, prec, nsteps + 1, dt),
               elements=s.n_hex + s.n_prism + s.n_tet + s.n_pyr, n_hex=s.n_hex, n_prism=s.n_prism, dof=s.n_state,
               ms_per_step=wall * 1e3 / nsteps, p50_step_ms=float(np.percentile(per, 50)),
               p99_step_ms=float(np.percentile(per, 99)),
               gdof_rhs_s=s.n_state * 4 * nsteps / wall / 1e9, finite=finite,
               conservation_drift=[float(x) for x in (c1 - c0) / scale], domain_volume=vol)
    del s, st
    torch.cuda.empty_cache()
    return out


def serving_dt(n, p, kind, u0=1.0, c0=10.0):
    """RK4 step of a serving request: 0.25 h / ((2p+1)(U0 + c0)), h the cell
    size, c0 = 1/Ma (the same bound for hexahedra and prisms; twice this
    step is unstable on hexahedra)."""
    h = 2 * np.pi / n
    return 0.25 * h / ((2 * p + 1) * (u0 + c0))


def run_serving(frmi, torch, budget_gib=64.0, max_active=64, nreq=512, seed=0, check_every=64):
    """The serving stream: requests arrive by their Poisson schedule (wall
    clock), are queued, admitted by device footprint and slot limit, and
    advanced together one RK4 step per pool round until done.  Step latency
    = wall time of one pool round that advanced at least one request."""
    from paper_2401_06132_amd import inputs
    reqs = inputs.serving_requests(n=nreq, seed=seed)
    budget = int(budget_gib * (1 << 30))
    pool = frmi.Pool(budget, max_active=max_active, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0)
    outs, t_arr, t_adm, t_fin, dof_req = {}, {}, {}, {}, {}
    step_ms, step_dof, active, launches = [], [], [], []
    peak_bytes, nxt, done, work = 0, 0, 0, 0
    t0 = time.perf_counter()
    last_print = t0
    while done < nreq:
        now = time.perf_counter() - t0
        while nxt < nreq and reqs[nxt]["arrival"] <= now:
            r = reqs[nxt]
            kw = dict(n=r["n"], p=r["p"], kind=r["etype"], nsteps=r["steps"],
                      dt=serving_dt(r["n"], r["p"], r["etype"]), tgv_p0=inputs.P0)
            if r["id"] % check_every == 0:
                kw["u_out"] = np.empty(pool.footprint(**kw)[1])
            rid = pool.submit(**kw)
            if "u_out" in kw:
                outs[rid] = kw["u_out"]
            t_arr[rid] = r["arrival"]
            dof_req[rid] = pool.footprint(**kw)[1]
            nxt += 1
        ts = time.perf_counter()
        st, adm, fin = pool.step()
        te = time.perf_counter()
        for i in adm:
            t_adm[i] = te - t0
        for i in fin:
            t_fin[i] = te - t0
        done += len(fin)
        peak_bytes = max(peak_bytes, st["bytes_in_use"])
        if st["n_active"] > 0:
            step_ms.append((te - ts) * 1e3)
            step_dof.append(st["dof"])
            active.append(st["n_active"])
            launches.append(st["n_launches"])
            work += 4 * st["dof"]
        elif st["n_queued"] == 0 and not adm and nxt < nreq:
            time.sleep(max(0.0, reqs[nxt]["arrival"] - (time.perf_counter() - t0)))
        if te - last_print > 10:
            last_print = te
            print("serving: t=%.1fs done=%d submitted=%d active=%d queued=%d" %
                  (te - t0, done, nxt, st["n_active"], st["n_queued"]), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    lat = np.array([t_fin[i] - t_arr[i] for i in t_fin])
    wait = np.array([t_adm[i] - t_arr[i] for i in t_adm])
    finite = all(bool(np.isfinite(o).all()) for o in outs.values())
    sm = np.array(step_ms)
    return {
        "workload": "%d Taylor-Green requests, Poisson arrivals (mean %.0f/s), n^3 boxes n in 6..32, hex|prism, "
                    "p in {2,3,4}, 20-200 RK4 steps, fp32 fused" % (nreq, 200.0),
        "budget_GiB": budget_gib, "max_active": max_active, "requests": nreq, "wall_s": wall,
        "rounds": len(step_ms), "p50_step_ms": float(np.percentile(sm, 50)),
        "p99_step_ms": float(np.percentile(sm, 99)), "max_step_ms": float(sm.max()),
        "gdof_rhs_s": work / wall / 1e9, "gdof_rhs_s_busy": work / (sm.sum() * 1e-3) / 1e9,
        "mean_active": float(np.mean(active)), "max_active_seen": int(max(active)),
        "mean_launches_per_step": float(np.mean(launches)), "peak_GiB": peak_bytes / (1 << 30),
        "p50_request_latency_s": float(np.percentile(lat, 50)), "p99_request_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_wait_s": float(np.percentile(wait, 50)), "p99_queue_wait_s": float(np.percentile(wait, 99)),
        "checked_finite": len(outs), "finite": finite,
    }


def cpu_baseline(budget_s=20.0):
    """The oracle (plain NumPy, dense operators) on the host: one RHS of the
    same Taylor-Green hex p=3 workload on a smaller periodic box; the box is
    chosen so that the run takes roughly budget_s seconds."""
    from oracle.mesh import Mesh
    from oracle.rhs import Params, rhs
    from paper_2401_06132_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    def run(N):
        m = Mesh(N, N, N, 3, "hex")
        U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
        t0 = time.perf_counter()
        rhs(m, U, Params(pref=inputs.P0))
        return time.perf_counter() - t0, 5 * m.nelem["hex"] * m.refs["hex"].nu

    # an 8^3 probe sizes the sample box for about budget_s of work
    t8, _ = run(8)
    N = int(max(8, min(32, round(8 * (budget_s / max(t8, 1e-3)) ** (1.0 / 3.0)))))
    elapsed, dof = run(N)
    return {"value": dof / elapsed / 1e9, "unit": "GDoF-RHS/s", "cores": int(threads), "kind": "oracle",
            "sample": "one RHS of the TGV hex p=3 flux-AA case on a %d^3 periodic box (%d DoF), %.2f s" %
                      (N, dof, elapsed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline variant only")
    ap.add_argument("--only", default=None, help="one variant kind:prec:p:form, e.g. prism:fp32:3:fused (profiling)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-only", action="store_true", help="only the serving stream")
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2401_06132_amd as frmi
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "copies": 3}))
        return
    if args.serving_only:
        sv = run_serving(frmi, torch, args.serving_budget_gib, args.serving_slots, args.serving_requests)
        print(json.dumps({"serving": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sv.items()}}),
              flush=True)
        return
    variants = {}
    if args.only:
        kind, prec, p, form = args.only.split(":")
        r = time_variant(frmi, torch, args.n, int(p), prec, args.steps, args.warmup, form, kind)
        r["gdof_s"] = r["n_dof"] * args.steps / r["wall_s"] / 1e9
        print(json.dumps({"variant": args.only, **{k: (round(v, 4) if isinstance(v, float) else v)
                                                   for k, v in r.items()}}), flush=True)
        return
    order = [("fp32", 3, "fused", "hex")] if args.quick else [
        ("fp32", 3, "fused", "hex"), ("fp64", 3, "fused", "hex"), ("fp64", 3, "plain", "hex"),
        ("fp32", 4, "fused", "hex"), ("fp64", 4, "fused", "hex"), ("fp64", 4, "plain", "hex"),
        ("fp32", 3, "fused", "prism"), ("fp64", 3, "fused", "prism"), ("fp64", 3, "plain", "prism"),
        ("fp32", 4, "fused", "prism"),
        ("fp32", 3, "noaa", "hex"), ("fp64", 3, "noaa", "hex"), ("fp32", 4, "noaa", "hex"),
        ("fp32", 3, "noaa", "prism"), ("fp32", 4, "noaa", "prism"),
        ("fp32", 3, "fullaa", "hex"), ("fp64", 3, "fullaa", "hex"), ("fp32", 4, "fullaa", "hex"),
        ("fp64", 4, "fullaa", "hex"), ("fp32", 3, "fullaa", "prism"), ("fp32", 4, "fullaa", "prism"),
        ("fp32", 3, "fused", "tet"), ("fp64", 3, "fused", "tet"), ("fp32", 4, "fused", "tet"),
        ("fp32", 3, "noaa", "tet"), ("fp32", 4, "noaa", "tet"), ("fp64", 3, "plain", "tet"),
        ("fp32", 3, "fused", "pyr"), ("fp64", 3, "fused", "pyr"), ("fp32", 4, "fused", "pyr"),
        ("fp32", 3, "noaa", "pyr"), ("fp64", 3, "plain", "pyr"), ("fp32", 3, "fused", "hex_pyr"),
        ("fp32", 3, "fused", "hex_pyr_tet"), ("fp32", 3, "fused", "hex_prism_pyr_tet"),
        ("fp32", 3, "fused", "hex_warp"), ("fp64", 3, "fused", "hex_warp"), ("fp32", 4, "fused", "hex_warp"),
        ("fp32", 3, "fused", "prism_warp"), ("fp32", 4, "fused", "prism_warp")]
    for prec, p, form, kind in order:
        ksteps = args.steps if kind == "hex" else max(5, args.steps // 3)
        r = time_variant(frmi, torch, args.n, p, prec, ksteps, args.warmup, form, kind)
        br = 4 if prec == "fp32" else 8
        vb, vf = volume_model(p, br)
        E = r["n_elem"]
        r["gdof_s"] = r["n_dof"] * ksteps / r["wall_s"] / 1e9
        if kind == "hex":
            r["vol_GBs"] = vb * E / (r["vol_ms"] * 1e-3) / 1e9
            r["vol_TFLOPs"] = vf * E / (r["vol_ms"] * 1e-3) / 1e12 if form == "fused" else float("nan")
            r["rhs_GBs"] = rhs_bytes_model(p, br) * E * ksteps / r["wall_s"] / 1e9
        else:
            r["vol_GBs"] = r["vol_TFLOPs"] = r["rhs_GBs"] = float("nan")
        variants["%s%s%s_p%d" % ("" if kind == "hex" else kind + "_", "" if form == "fused" else form + "_", prec,
                                  p)] = r
        print("variant", form, prec, p, json.dumps({k: round(v, 4) if isinstance(v, float) else v for k, v in r.items()}),
              file=sys.stderr, flush=True)
    head = variants["fp32_p3"]
    for pre in ("", "prism_"):
        for p in (3, 4):
            a, b = "%sfp32_p%d" % (pre, p), "%splain_fp64_p%d" % (pre, p)
            if a in variants and b in variants:
                variants[a]["speedup_vs_plain_fp64"] = variants[a]["gdof_s"] / variants[b]["gdof_s"]
    vb, vf = volume_model(3, 4)
    ai = vf / vb
    ridge = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai > ridge:
        roof = {"bound": "alu", "achieved": round(head["vol_TFLOPs"], 3), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(head["vol_TFLOPs"] / VALU_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(head["vol_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(head["vol_GBs"] / HBM_PEAK_GBS, 4)}
    traffic = HEX_VOL_P3_FP32_TRAFFIC if args.n == 48 else None
    roof.update({"kernel": "hex_volume<3,float>", "traffic": traffic, "traffic_unit": "bytes per launch",
                 "algorithmic_bytes": vb * head["n_elem"], "hbm_GBs": round(head["vol_GBs"], 1),
                 "hbm_frac": round(head["vol_GBs"] / HBM_PEAK_GBS, 4), "flop_per_byte": round(ai, 2),
                 "avg_ms": round(head["vol_ms"], 4)})
    def _r(x):
        return round(x, 4) if isinstance(x, float) and np.isfinite(x) else (x if not isinstance(x, float) else None)
    out = {
        "metric": METRIC, "value": round(head["gdof_s"], 3), "unit": "GDoF-RHS/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Taylor-Green vortex, %d^3 periodic hex, p=3, flux AA GL(6)^3, fused, FP32 bulk / "
                               "FP64 state" % args.n, "elements": head["n_elem"], "dof": head["n_dof"]},
        "p50_step_ms": round(head["p50_ms"], 4), "p99_step_ms": round(head["p99_ms"], 4),
        "hbm_frac_rhs": round(head["rhs_GBs"] / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "variants": {k: {"gdof_s": _r(v["gdof_s"]), "p99_step_ms": _r(v["p99_ms"]), "vol_ms": _r(v["vol_ms"]),
                         "hbm_frac_rhs": _r(v["rhs_GBs"] / HBM_PEAK_GBS), "finite": v["finite"],
                         "speedup_vs_plain_fp64": _r(v.get("speedup_vs_plain_fp64", float("nan")))}
                     for k, v in variants.items()},
    }
    if not args.quick:
        rk = run_rk(frmi, torch, "mixed", 64, 4, "fp32", 99, 2e-4)
        out["mixed_rk4"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rk.items()}
        print("mixed rk4", json.dumps(out["mixed_rk4"]), file=sys.stderr, flush=True)
    if not args.quick and not args.no_serving:
        sv = run_serving(frmi, torch, args.serving_budget_gib, args.serving_slots, args.serving_requests)
        out["serving"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sv.items()}
        print("serving", json.dumps(out["serving"]), file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
