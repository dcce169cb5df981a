"""Benchmark of the arrested-Newton-flow hot path on one MI355X.

Workload (default): the large Ginzburg-Landau lattice, 4096 x 4096 interior
sites, kappa = 1.5 (lambda = 2 kappa^2 = 4.5), h = 0.2, 256 unit vortices at
seeded Poisson-disc positions (minimum separation 3) inside the centred square
of side 0.6 L, U(+-1e-3) noise, FP32 fields with FP64 reductions. A "step" is
one full step of arrested Newton flow. By default it is integrated by velocity
Verlet in one pass per step (read phi, v and the stored force, write the new
ones, reduce the new field's FP64 energy for the arrest test of eq. (4)); with
--integrator rk4 it is one classical RK4 step (the first stage pass with the
energy and arrest test, then one fused pass for stages 2-4 or three separate
stage passes, whichever plan the autotuner picks); --integrator gf times plain
gradient flow.

Prints one JSON line: site-updates/s over K timed steps (inputs resident in
HBM), the roofline of the dominant pass (algorithmic bytes per launch over its
mean HIP-event duration), and the CPU oracle's rate on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM traffic of each pass, in field sets (C planes) read and
# written per interior site (halo re-reads served by cache are not counted):
#   P1 reads phi, writes a1; P2 reads phi, v, writes a2; P3 reads phi, v, a1, a2,
#   writes q; P4 reads phi, v, a2, q, a1, writes phi', v'.
#   P234 (fused stages 2-4) reads phi, v, a1, writes phi', v'.
#   VV (velocity Verlet, one pass) reads phi, v, a, writes phi', v', a';
#   GF (gradient flow, one pass) reads phi, a, writes phi', a'.
# field sets (C components of one lattice) read and written per launch; velocity
# Verlet in kick-drift-kick form (VV) reads phi and u and writes phi' and u', in
# its stored-force form (VVA) reads phi, v, a and writes phi', v', a'; gradient
# flow on the lattice theories (GF) reads phi and writes phi'
PASS_SETS = {"P1": (1, 1), "P2": (2, 1), "P3": (4, 1), "P4": (5, 2), "P234": (3, 2), "VV": (2, 2), "VVA": (3, 3),
             "GF": (1, 1)}
STEP_SETS = 17          # separate stage passes
STEP_SETS_FUSED = 7     # P1 + fused stages 2-4
PLAN_NAMES = ["stages", "fused"]

WORKLOADS = {
    "gl4096": dict(theory="abelian_higgs", N=4096, h=0.2, kappa=1.5, nv=256, seed=4, dtype="f32"),
    "cm512": dict(theory="chiral_magnet", N=512, h=0.05, seed=2, dtype="f32"),
    "ah128": dict(theory="abelian_higgs", N=128, h=0.1, kappa=2 ** -0.5, nv=1, seed=1, dtype="f64"),
    "batch256": dict(theory="abelian_higgs", n=256, base_seed=3000, h=0.2, dtype="f32"),
    "unet256": dict(levels=4, base=32, cin=2, cout=4, N=8, H=256, W=256),
    # the other theories (context lines, with their own step models below)
    "heusler_demag512": dict(theory="chiral_magnet", N=512, h=0.05, dtype="f32", integrator="vv", seed=5,
                             params=[1.0, 1.0, 2.0, 0.0, 1.057], dmi="heusler", demag=True),
    "bec256": dict(theory="bec", N=256, h=0.1, dtype="f32", integrator="rk4", seed=6, params=[0.038, 0.99, 1000.0]),
    # the Skyrme term stiffens the flow where |grad m| is large: C = 0.25 keeps dt^2 times the
    # largest stiffness below the velocity Verlet limit for this skyrmion size
    "bs512": dict(theory="baby_skyrme", N=512, h=0.1, dtype="f32", integrator="vv", seed=7, params=[1.0, 0.1, 0.25]),
}

BF16_DENSE_PEAK_TFLOPS = 2500.0


def unet_step_bytes(wl):
    """Bytes one training step of the U-Net reads and writes in its activation
    tensors (BF16), layer by layer, per pixel of the layer's level: forward reads
    the input (C_in) and writes the pre-activation and the activation (2 C_out);
    backward reads the output gradient and the pre-activation (2 C_out) and the input
    (C_in) and writes the input gradient (C_in); the weight gradient reads the
    input and the output gradient again (C_in + C_out). Weights, pooling,
    upsampling and the head are small beside these and are left out."""
    from paper_2603_24370_amd.learned import unet_param_shapes
    total = 0
    for name, shp in unet_param_shapes(wl["levels"], wl["base"], wl["cin"], wl["cout"]):
        if not name.endswith(".w") or len(shp) != 4:
            continue
        cout, cin = shp[0], shp[3]
        level = 0 if name.startswith("head") else int(name[3]) if name[:3] in ("enc", "dec") else wl["levels"] - 1
        pixels = wl["N"] * (wl["H"] >> level) * (wl["W"] >> level)
        total += pixels * 2 * ((cin + 2 * cout) + (2 * cout + 2 * cin) + (cin + cout))
    return total


def unet_roofline(tflops, step_bytes, step_flops, step_s, infer_tflops):
    """Roofline of the U-Net training step. Its arithmetic intensity (flops over the
    activation bytes of unet_step_bytes) lies below the BF16 ridge (2.5 PFLOP/s over
    8 TB/s = 312 flop/B), so HBM bounds it: achieved = those bytes over the step
    time, against 8 TB/s."""
    intensity = step_flops / step_bytes
    gbps = step_bytes / step_s / 1e9
    ridge = BF16_DENSE_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    bound = "hbm" if intensity < ridge else "mfma"
    if bound == "hbm":
        ach, peak, unit = gbps, HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = tflops, BF16_DENSE_PEAK_TFLOPS, "TFLOP/s"
    return {"bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit, "frac": round(ach / peak, 4),
            "traffic": None, "kernel": "conv3x3_tiled + conv3x3_mfma + conv3x3_wgrad (whole training step)",
            "intensity_flop_per_B": round(intensity, 1), "ridge_flop_per_B": round(ridge, 1),
            "TFLOPs": round(tflops, 2), "frac_of_bf16_peak": round(tflops / BF16_DENSE_PEAK_TFLOPS, 4),
            "step_GB": round(step_bytes / 1e9, 4), "inference_TFLOPs": round(infer_tflops, 2)}


def run_unet(args, wl):
    """Training throughput of the learned initialiser's U-Net (BF16 MFMA, FP32
    accumulate): forward + backward + Adam on batches of 8 images of 256^2."""
    import numpy as np
    import torch
    import paper_2603_24370_amd as ss
    net = ss.Net(wl["levels"], wl["base"], wl["cin"], wl["cout"], wl["N"], wl["H"], wl["W"])
    rng = np.random.default_rng(0)
    # He-uniform weights, zero biases, in the exchange order
    from paper_2603_24370_amd.learned import unet_param_shapes
    flat = []
    for name, shp in unet_param_shapes(wl["levels"], wl["base"], wl["cin"], wl["cout"]):
        if name.endswith(".b"):
            flat.append(np.zeros(int(np.prod(shp))))
        else:
            lim = np.sqrt(6.0 / int(np.prod(shp[1:])))
            flat.append(rng.uniform(-lim, lim, size=int(np.prod(shp))))
    net.set_weights(np.concatenate(flat).astype(np.float32))
    x = torch.randn((wl["N"], wl["H"], wl["W"], wl["cin"]), device="cuda:0")
    t = torch.randn((wl["N"], wl["H"], wl["W"], wl["cout"]), device="cuda:0")
    for _ in range(args.warmup):
        net.train_step(x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    f_fwd, f_bwd = net.flops()
    tfl = args.steps * wl["N"] * (f_fwd + f_bwd) / el / 1e12
    step_bytes = unet_step_bytes(wl)
    # inference alone
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(x)
    torch.cuda.synchronize()
    el_f = time.perf_counter() - t1
    tfl_f = args.steps * wl["N"] * f_fwd / el_f / 1e12
    out = {"metric": "training images/s", "value": args.steps * wl["N"] / el, "unit": "images/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)",
           "data": "synthetic", "config": {"workload": "unet256", **wl},
           "roofline": unet_roofline(tfl, step_bytes, wl["N"] * (f_fwd + f_bwd), el / args.steps, tfl_f),
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    net.close()


def other_theory_bytes(name, wl, demag_iters=2, nlev=1, half_step=False):
    """Bytes per interior site and step that the kernels of a step read and write
    (FP32 fields, FP64 solver planes; halo re-reads not counted):
      heusler_demag512, velocity Verlet: the pass reads phi, v, a and writes phi', v',
        a' (6 x 3 x 4 B; in the half-step form phi and u in and out, 4 x 3 x 4 B); the
        solve forms the stage point (reads 3 sets, writes one: 48 B; half-step form
        2 and one, 36 B), starts conjugate gradients (reads S_1, S_2 and x, writes r,
        rhs, psi: 40 B) and per iteration moves about 210 B on the lattice (the V-cycle's
        three launches on level 0 70 B: pre-smoothing reads psi and rhs and writes tmp,
        the restriction reads tmp and rhs, post-smoothing reads tmp, rhs and the coarse
        correction and writes psi; the coarser levels a third of that; the
        conjugate-gradient kernels 120 B);
      bec256, RK4 with the atom-number constraint: stage points 104 B, gradients 64 B,
        forces and updates 152 B, the end-of-step scaling 32 B (two components);
      bs512, velocity Verlet: 6 x 3 x 4 B (half-step form 4 x 3 x 4 B).
    The half-step form's restart pass after an arrest (reads phi, writes u) is not
    counted."""
    if name == "heusler_demag512":
        return (48 + 36 if half_step else 72 + 48) + 40 + demag_iters * 210
    if name == "bec256":
        return 352
    return 48 if half_step else 72


def run_other(args, name, wl):
    """A flow of one of the other theories, timed over graph replays of ss_minimise
    (no stop rule fires: grad_tol = 0, max_steps = warm-up + steps)."""
    import torch
    import paper_2603_24370_amd as ss
    N, h = wl["N"], wl["h"]
    kw = {}
    if wl.get("demag") or wl.get("dmi", "bulk") != "bulk":
        kw = {"dmi": wl.get("dmi", "bulk"), "demag": wl.get("demag", False)}
    s = ss.Solver(wl["theory"], N, N, h, wl["params"], dtype=wl["dtype"], **kw)
    s.set_integrator(wl["integrator"])
    if wl["theory"] == "bec":
        R = 7.0  # about the Thomas-Fermi radius of these parameters
        cen = [(2.0 * math.cos(k * math.pi / 3), 2.0 * math.sin(k * math.pi / 3)) for k in range(6)]
        s.init_bec(R=R, xi=0.5, centres=cen, seed=wl["seed"], noise_amp=0.05)
    elif wl.get("dmi") == "heusler":
        s.init_skyrmion(R=0.6, gamma=-math.pi / 2, seed=wl["seed"], noise_amp=1e-3, vorticity=-1)
    else:
        s.init_skyrmion(R=2.0, gamma=0.0, seed=wl["seed"], noise_amp=1e-3)
    s.minimise(grad_tol=0.0, max_steps=args.warmup, graph_steps=16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = s.minimise(grad_tol=0.0, max_steps=args.warmup + args.steps, graph_steps=16)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    done = res["step"] - args.warmup
    sites = N * N
    ms_step = 1e3 * el / max(done, 1)
    half = wl["integrator"] == "vv" and s.vv_form == ss.SS_VV_HALF_STEP
    per_site = other_theory_bytes(name, wl, half_step=half)
    gbps = per_site * sites / (ms_step * 1e-3) / 1e9
    obs = s.observables()
    out = {"metric": "site-updates/s", "value": sites * done / el, "unit": "site-updates/s", "n_gpus": 1,
           "steps": done, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 fields, f64 reductions" + (
               " and f64 solver" if wl.get("demag") else ""),
           "data": "synthetic (seeded ansatz + noise)",
           "config": {"workload": name, "theory": wl["theory"], "Nx": N, "Ny": N, "h": h, "params": wl["params"],
                      "dmi": wl.get("dmi"), "demag": wl.get("demag", False),
                      "integrator": INTEGRATOR_NAMES[wl["integrator"]], "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "whole step (every kernel of the step; bytes per site from the step model)",
                        "step_bytes_per_site": per_site},
           "cpu_baseline": None,
           "state": {"energy": obs["energy"], "step": res["step"], "n_arrests": res["n_arrests"],
                     "atoms": obs.get("atoms"), "q_bl": obs.get("q_bl")}}
    print(json.dumps(out), flush=True)
    s.close()


def run_batch(args, wl):
    """256 independent GL lattices (sides 64..384, kappa 0.5..2, 1..8 vortices)
    advanced by batched launches (one launch per pass for all members)."""
    import torch
    import paper_2603_24370_amd as ss
    from paper_2603_24370_amd import inputs as I
    insts = [I.gl_batch_instance(b, wl["base_seed"], wl["h"]) for b in range(wl["n"])]
    B = ss.Batch("abelian_higgs", [(m.Nx, m.Ny, m.h, m.params) for m in insts], dtype=wl["dtype"])
    B.set_integrator(args.integrator)
    tune = B.autotune(args.autotune_steps) if args.autotune_steps else None
    for m, mem in zip(insts, B.members):
        mem.init_vortices(m.centres, seed=m.seed, noise_amp=1e-3)
    sites = sum(m.Nx * m.Ny for m in insts)
    B.flow_step(args.warmup, want_info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.flow_step(args.steps, want_info=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / args.steps
    batch_plan = B.plan
    one_pass = args.integrator != "rk4"
    if one_pass:
        step_sets = sum(PASS_SETS[args.integrator.upper()])
        kname = f"batch_pass ({args.integrator.upper()} step)"
    else:
        step_sets = STEP_SETS_FUSED if batch_plan == 1 else STEP_SETS
        kname = ("batch_pass + batch_pass_fused (whole step)" if step_sets == STEP_SETS_FUSED
                 else "batch_pass (whole step)")
    step_gbps = step_sets * 4 * 4 * sites / (ms_step * 1e-3) / 1e9
    out = {"metric": "site-updates/s", "value": sites * args.steps / el, "unit": "site-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 fields, f64 reductions",
           "data": "synthetic (seeded ansatz + noise)",
           "config": {"workload": "batch256", "members": wl["n"], "interior_sites": sites, "h": wl["h"],
                      "grad_form": "euler-lagrange", "integrator": INTEGRATOR_NAMES[args.integrator],
                      "parallelism": "single GPU, one launch per pass"},
           "roofline": {"bound": "hbm", "achieved": round(step_gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(step_gbps / HBM_PEAK_GBS, 4), "traffic": None, "step_sets": step_sets,
                        "kernel": kname},
           "tile": {"chosen": list(ss_tile(tune[0])) if tune else None,
                    "plan": "one pass" if one_pass else PLAN_NAMES[batch_plan],
                    "step_ms_by_plan_and_tile": {PLAN_NAMES[p]: [round(x, 4) for x in row]
                                                 for p, row in enumerate(tune[2])} if tune else None},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    B.close()


CONVERGE_CASES = [
    # (name, theory, N, h, params, grad_mode, integrator, courant, grad_tol)
    ("ah128 EL", "abelian_higgs", 128, 0.1, [1.0], 0, "rk4", 0.5, 1e-6),
    ("ah128 EL", "abelian_higgs", 128, 0.1, [1.0], 0, "vv", 0.5, 1e-6),
    ("ah128 EL", "abelian_higgs", 128, 0.1, [1.0], 0, "gf", 0.5, 1e-6),
    ("ah128 EL", "abelian_higgs", 128, 0.1, [1.0], 0, "gf", 0.6, 1e-6),
    ("cm128 EL", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 0, "rk4", 0.5, 1e-6),
    ("cm128 EL", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 0, "vv", 0.5, 1e-6),
    ("cm128 EL", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 0, "gf", 0.5, 1e-6),
    ("cm128 exact", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 1, "rk4", 0.5, 1e-6),
    ("cm128 exact", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 1, "vv", 0.5, 1e-6),
    ("cm128 exact", "chiral_magnet", 128, 0.1, [1.0, 1.0, 0.1, 0.6], 1, "gf", 0.5, 1e-6),
]


def run_converge(args):
    """Flow steps and wall time to ||G||_inf < tol (FP64) for each integrator:
    the critical vortex of 128^2 at h = 0.1 (one vortex at the origin, seeded noise
    1e-3, seed 1) and a Belavin-Polyakov skyrmion of radius 2 on 128^2 at h = 0.1
    (seed 2) with both gradient forms. Tests whether the arrested second-order flow
    beats first-order descent (gradient flow with tau = (C h)^2 / 2)."""
    import torch
    import paper_2603_24370_amd as ss
    rows = []
    for name, theory, N, h, params, gm, integ, C, tol in CONVERGE_CASES:
        s = ss.Solver(theory, N, N, h, params, dtype="f64", grad_mode=gm, courant=C)
        s.set_integrator(integ)
        if theory == "abelian_higgs":
            s.init_vortices([(0.0, 0.0)], seed=1, noise_amp=1e-3)
        else:
            s.init_skyrmion(R=2.0, gamma=-math.pi / 2, seed=2, noise_amp=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = s.minimise(grad_tol=tol, max_steps=args.converge_max_steps, graph_steps=64)
        el = time.perf_counter() - t0
        obs = s.observables()
        rows.append({"case": name, "integrator": integ, "courant": C, "steps": res["step"],
                     "arrests": res["n_arrests"], "reason": res["reason"], "gnorm_inf": res["gnorm_inf"],
                     "energy": res["energy"], "wall_s": round(el, 3),
                     "q": obs["n_wind"] if theory == "abelian_higgs" else obs["q_bl"]})
        print(json.dumps(rows[-1]), flush=True)
        s.close()
    out = {"metric": "flow steps and wall time to ||G||_inf < 1e-6", "value": None, "unit": "s", "n_gpus": 1,
           "steps": None, "warmup": 0, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic (seeded ansatz + noise)",
           "config": {"workload": "converge", "max_steps": args.converge_max_steps}, "results": rows,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def ss_tile(i):
    import paper_2603_24370_amd as ss
    return ss.ss_tile_shape(i)


STAGE_SOURCES = ["ss_internal.hpp", "ss_theory.hpp", "ss_kernels.hpp", "ss_api.hip"]


def _code_only(text: str) -> str:
    """C++ source without comments and blank lines (a comment edit leaves the
    kernels, and so their counters, unchanged)."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] in "\"'":
            j = i + 1
            while j < n and text[j] != text[i]:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def kernel_source_hash() -> str:
    """Hash of the code (comments stripped) the stage kernels are built from
    (traffic counters taken on other code are not reported)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_24370_amd", "csrc")
    for f in STAGE_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


INTEGRATOR_NAMES = {"rk4": "RK4 arrested Newton flow, dt = 0.5 h",
                    "vv": "velocity Verlet arrested Newton flow (one pass per step), dt = 0.5 h",
                    "gf": "gradient flow (one pass per step), tau = dt^2 / 2, dt = 0.5 h"}


def make_solver(wl, autotune_steps=10, integrator="rk4", grad="el"):
    import paper_2603_24370_amd as ss
    from paper_2603_24370_amd import inputs as I
    tune = None
    gm = ss.SS_GRAD_EXACT if grad == "exact" else ss.SS_GRAD_EL
    if wl["theory"] == "abelian_higgs":
        lam = I.gl_lambda_from_kappa(wl["kappa"])
        s = ss.Solver("abelian_higgs", wl["N"], wl["N"], wl["h"], [lam], dtype=wl["dtype"], grad_mode=gm)
        s.set_integrator(integrator)
        if autotune_steps:
            tune = s.autotune(autotune_steps)
        if wl["nv"] == 1:
            centres = [(0.0, 0.0)]
        else:
            centres = I.poisson_disc(wl["seed"], wl["nv"], 3.0, 0.5 * 0.6 * wl["N"] * wl["h"])
        s.init_vortices(centres, seed=wl["seed"], noise_amp=1e-3)
        params = [lam]
    else:
        params = [1.0, 1.0, 0.1, 0.6]
        s = ss.Solver("chiral_magnet", wl["N"], wl["N"], wl["h"], params, dtype=wl["dtype"], grad_mode=gm)
        s.set_integrator(integrator)
        if autotune_steps:
            tune = s.autotune(autotune_steps)
        s.init_skyrmion(R=2.0, gamma=-math.pi / 2, seed=wl["seed"], noise_amp=1e-3)
    return s, params, tune


def host_cores() -> int:
    """Cores this process may use: its CPU affinity, capped by OMP_NUM_THREADS
    where set (the host's share for one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(s, wl, params, window=1024, steps=None, scheme="rk4", target_s=3.0, grad="el"):
    """The FP64 oracle as it stands (one thread per call) on windows of the same
    field: first one core on the central window, then every usable host core at
    once, one window per thread (the oracle is a C library called through
    ctypes, which releases the interpreter lock, so the threads run in parallel).
    Each window keeps its neighbours as a fixed halo. Without a step count, two
    calibration steps set it so that the one-core run takes about target_s."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.build(force=False)
    f = s.get_field().double().cpu().numpy()
    N = wl["N"]
    w = min(window, N)

    def window_at(a, b):
        return np.ascontiguousarray(f[:, a:a + w + 4, b:b + w + 4])

    mode = oracle.GRAD_EXACT if grad == "exact" else oracle.GRAD_EL

    def run(sub):
        oracle.flow(wl["theory"], sub, np.zeros_like(sub), wl["h"], params, steps, scheme=scheme, mode=mode)

    c = (N - w) // 2
    if steps is None:
        t0 = time.perf_counter()
        oracle.flow(wl["theory"], window_at(c, c), np.zeros_like(window_at(c, c)), wl["h"], params, 2,
                    scheme=scheme, mode=mode)
        steps = int(min(100000, max(10, math.ceil(target_s / max((time.perf_counter() - t0) / 2, 1e-9)))))
    t0 = time.perf_counter()
    run(window_at(c, c))
    dt1 = time.perf_counter() - t0
    cores = host_cores()
    per = max(1, N // w)
    origins = [((k // per) % per * w, k % per * w) for k in range(cores)]
    subs = [window_at(min(a, N - w), min(b, N - w)) for a, b in origins]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(run, subs))
    dtn = time.perf_counter() - t0
    return {"value": cores * w * w * steps / dtn, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} threads, each {steps} {scheme} steps of its own {w}x{w} window of the same field (its "
                      f"neighbours as a fixed halo), FP64, {dtn:.1f} s wall",
            "value_1core": w * w * steps / dt1,
            "sample_1core": f"{steps} {scheme} steps of the central {w}x{w} window on one core, {dt1:.1f} s"}


def measured_copy_gbps(nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device-to-device copy (read + write bytes over the
    mean time of `reps` copies of nbytes, HIP events): the practical ceiling
    a streaming kernel is also compared with."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def traffic_record(pass_name, wl_name, tile):
    """HBM bytes per launch of a pass on a tile shape (index) from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source") != kernel_source_hash():
        return None
    return rec.get(wl_name, {}).get(f"tile{tile}", {}).get(pass_name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="gl4096", choices=sorted(WORKLOADS) + ["converge"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--timing-steps", type=int, default=20)
    ap.add_argument("--autotune-steps", type=int, default=10, help="0 = keep the default tile shape")
    ap.add_argument("--converge-max-steps", type=int, default=400000)
    ap.add_argument("--grad", default="el", choices=["el", "exact"],
                    help="gradient form: the Euler-Lagrange expression (default) or the exact h^-2 dE_h/dphi")
    ap.add_argument("--integrator", default="vv", choices=sorted(INTEGRATOR_NAMES),
                    help="vv (velocity Verlet arrested Newton flow, default), rk4 (RK4 arrested Newton flow) or "
                         "gf (gradient flow)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times), to scale HBM counters")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "repeats": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the lattice fits one "
              f"MI355X; see the design notes for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "converge":
        run_converge(args)
        return
    wl = WORKLOADS[args.workload]
    if args.workload in ("heusler_demag512", "bec256", "bs512"):
        run_other(args, args.workload, wl)
        return
    if args.workload.startswith("batch"):
        run_batch(args, wl)
        return
    if args.workload.startswith("unet"):
        run_unet(args, wl)
        return
    s, params, tune = make_solver(wl, args.autotune_steps, args.integrator, args.grad)
    N = wl["N"]
    sites = N * N
    C = s.C
    b = 4 if wl["dtype"] == "f32" else 8

    # warm-up (real flow steps)
    s.flow_step(args.warmup, want_info=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.flow_step(args.steps, want_info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = s.info()
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    value = sites * args.steps / elapsed

    # per-pass device time with HIP events on the library's stream
    plan = s.plan
    ms = s.time_passes(args.timing_steps)
    import paper_2603_24370_amd as ss
    half_step = args.integrator == "vv" and s.vv_form == ss.SS_VV_HALF_STEP
    if args.integrator == "vv":
        names = ["VV" if half_step else "VVA"]
    elif args.integrator != "rk4":
        names = [args.integrator.upper()]
    else:
        names = ["P1", "P2", "P3", "P4"] if plan == 0 else ["P1", "P234"]
    passes = {}
    for k, name in enumerate(names):
        r, w_ = PASS_SETS[name]
        nbytes = sites * C * b * (r + w_)
        passes[name] = {"ms": ms[k], "GB_per_launch": nbytes / 1e9, "GBps": nbytes / (ms[k] * 1e-3) / 1e9}
    dom = max(passes, key=lambda k: passes[k]["ms"])
    ach = passes[dom]["GBps"]
    if half_step:
        # the restart pass that follows an arrest (reads phi, writes u): its mean
        # time per step, over steps where it works and steps where it returns at once
        st = s.info()
        passes["VV restart"] = {"ms": ms[1], "GB_per_launch": sites * C * b * 2 / 1e9,
                                "arrest_fraction": st["n_arrests"] / max(st["step"], 1)}
    if args.integrator != "rk4":
        step_sets = sum(PASS_SETS[names[0]])
    else:
        step_sets = STEP_SETS if plan == 0 else STEP_SETS_FUSED
    step_gbps = step_sets * C * b * sites / (ms_step * 1e-3) / 1e9
    # the counter record covers the Euler-Lagrange kernels only
    tr = traffic_record(dom, args.workload, ss.ss_get_tile(s.ctx)) if args.grad == "el" else None
    tr_gb = tr["total_GB"] if tr else None
    kname = {"P234": "stage_pass_fused (stages 2-4)", "VV": "stage_pass (velocity Verlet step, half-step form)",
             "VVA": "stage_pass (velocity Verlet step, stored force)",
             "GF": "stage_pass (gradient-flow step)"}.get(dom, f"stage_pass {dom}")
    if args.grad == "exact":
        kname = f"stage_pass_exact {dom}"
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr_gb, "traffic_unit": "GB per launch (rocprofv3 "
            "FETCH_SIZE x2 + WRITE_SIZE x1, scaled on a plain copy)", "traffic_over_algorithmic": tr["ratio"] if tr else None,
            "kernel": kname,
            "step_GBps": round(step_gbps, 1), "step_frac": round(step_gbps / HBM_PEAK_GBS, 4),
            "step_sets": step_sets,
            "passes": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in passes.items()}}

    copy = measured_copy_gbps()
    roof["copy_GBps"] = round(copy, 1)
    roof["frac_of_copy"] = round(ach / copy, 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(s, wl, params, scheme=args.integrator, grad=args.grad)

    out = {
        "metric": "site-updates/s",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields, f64 reductions" if wl["dtype"] == "f32" else "f64",
        "data": "synthetic (seeded ansatz + noise)",
        "config": {"workload": args.workload, "theory": wl["theory"], "Nx": N, "Ny": N, "h": wl["h"],
                   "kappa": wl.get("kappa"), "vortices": wl.get("nv"),
                   "grad_form": "euler-lagrange" if args.grad == "el" else "exact",
                   "integrator": INTEGRATOR_NAMES[args.integrator], "parallelism": "single GPU"},
        "roofline": roof,
        "tile": {"chosen": list(ss_tile(tune[0])) if tune else None,
                 "plan": PLAN_NAMES[plan] if args.integrator == "rk4" else "one pass",
                 "step_ms_by_plan_and_tile": {PLAN_NAMES[p]: [round(x, 4) for x in row]
                                              for p, row in enumerate(tune[2])} if tune else None},
        "cpu_baseline": cpu,
        "state": {"energy": info["energy"], "n_arrests": info["n_arrests"], "step": info["step"]},
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
