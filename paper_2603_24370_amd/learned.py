"""Learned initialiser for batched Ginzburg-Landau minimisations.

Pipeline (every arithmetic step runs in the library's HIP kernels):
  1. data: seeded instances (vortex centres, kappa) are relaxed by the batched
     arrested-Newton flow; the library turns each relaxed field into the
     network's target (smooth corrections to the vortex ansatz) and each
     instance into the network's input (vortex blob map, kappa);
  2. training: the BF16-MFMA U-Net minimises the mean squared error with Adam;
  3. use: input -> network -> ss_init_learned -> flow.
The plain ansatz start (ss_init_ansatz) remains the fallback and the baseline
of the comparison: both starts are flowed to the same reference energy and
their wall times are compared.
"""
from __future__ import annotations

import math
import time

import numpy as np

import paper_2603_24370_amd as ss
from paper_2603_24370_amd import inputs as I


def unet_param_shapes(levels=4, base=32, cin=2, cout=4):
    """(name, shape) of the network's parameters in the library's exchange order."""
    shapes = []
    ch = [base << l for l in range(levels)]
    c_prev = cin
    for l in range(levels - 1):
        shapes += [(f"enc{l}a.w", (ch[l], 3, 3, c_prev)), (f"enc{l}a.b", (ch[l],)),
                   (f"enc{l}b.w", (ch[l], 3, 3, ch[l])), (f"enc{l}b.b", (ch[l],))]
        c_prev = ch[l]
    L = levels - 1
    shapes += [("mid.a.w", (ch[L], 3, 3, c_prev)), ("mid.a.b", (ch[L],)),
               ("mid.b.w", (ch[L], 3, 3, ch[L])), ("mid.b.b", (ch[L],))]
    c_prev = ch[L]
    for l in reversed(range(levels - 1)):
        shapes += [(f"dec{l}a.w", (ch[l], 3, 3, c_prev + ch[l])), (f"dec{l}a.b", (ch[l],)),
                   (f"dec{l}b.w", (ch[l], 3, 3, ch[l])), (f"dec{l}b.b", (ch[l],))]
        c_prev = ch[l]
    shapes += [("head.w", (cout, c_prev)), ("head.b", (cout,))]
    return shapes


def init_weights(seed=0, levels=4, base=32, cin=2, cout=4):
    """He-uniform weights and zero biases as one flat fp32 array (exchange order)."""
    rng = np.random.default_rng(seed)
    flat = []
    for name, shp in unet_param_shapes(levels, base, cin, cout):
        k = int(np.prod(shp))
        if name.endswith(".b"):
            flat.append(np.zeros(k))
        else:
            lim = np.sqrt(6.0 / int(np.prod(shp[1:])))
            flat.append(rng.uniform(-lim, lim, size=k))
    return np.concatenate(flat).astype(np.float32)


def learned_instance(i: int, base_seed: int = 5_000_000, side: int = 256, h: float = 0.2) -> I.Instance:
    """Instance i of the learned-initialiser workload: the batched-GL distributions
    (kappa ~ U[0.5, 2], N ~ U{1..8}, centres uniform in the centred 0.6 L square)
    at a fixed side."""
    seed = base_seed + i
    u = I.uniform01(seed, I.STREAM_INSTANCE, np.arange(3, dtype=np.uint64))
    kappa = 0.5 + 1.5 * u[1]
    nv = 1 + min(int(u[2] * 8), 7)
    centres = I.uniform_centres(seed, nv, 0.5 * 0.6 * side * h)
    return I.Instance("abelian_higgs", side, side, h, [I.gl_lambda_from_kappa(kappa)], centres, seed, kappa=kappa)


def generate_dataset(insts, batch=64, rel_e_tol=0.0, window=0, max_steps=150, device="cuda:0", log=None):
    """Flow the instances with the batched solver (FP32 fields, FP64 reductions) for
    max_steps steps (or to the stall rule, if rel_e_tol > 0) and return
    (inputs (n, H, W, 2), targets (n, H, W, 4)) as fp32 device tensors.

    The default horizon of 150 steps relaxes the vortex cores (the fast modes:
    a single vortex reaches 1e-6 of its energy in about 100 steps) while the
    vortices have barely moved; later the field changes mainly by the slow drift
    of interacting vortices, which depends on all of them and would dominate
    the targets with values the network cannot infer from a blob map."""
    import torch
    n = len(insts)
    H, W = insts[0].Ny, insts[0].Nx
    X = torch.empty((n, H, W, 2), dtype=torch.float32, device=device)
    T = torch.empty((n, H, W, 4), dtype=torch.float32, device=device)
    stats = []
    for b0 in range(0, n, batch):
        chunk = insts[b0:b0 + batch]
        B = ss.Batch("abelian_higgs", [(m.Nx, m.Ny, m.h, m.params) for m in chunk], dtype="f32", device=device)
        for m, mem in zip(chunk, B.members):
            mem.init_vortices(m.centres, seed=m.seed, noise_amp=1e-3)
        rc, infos = B.minimise(grad_tol=0.0, rel_e_tol=rel_e_tol, window=window, max_steps=max_steps, graph_steps=16)
        for k, (m, mem) in enumerate(zip(chunk, B.members)):
            ss.ss_learned_input(mem.ctx, m.centres, m.kappa, X[b0 + k].data_ptr())
            ss.ss_learned_targets(mem.ctx, m.centres, None, T[b0 + k].data_ptr())
            stats.append(infos[k]["step"])
        B.close()
        if log:
            log(f"[data] {b0 + len(chunk)}/{n} relaxed (median steps {int(np.median(stats))})")
    return X, T, stats


def lr_at(step, total, lr, warmup=0, per_step=False, steps_per_epoch=1):
    """Learning rate of an Adam step: a linear warm-up over the first `warmup`
    steps, then a cosine decay from lr to 0, evaluated per step (per_step) or
    held constant within each epoch."""
    w = min(1.0, (step + 1) / warmup) if warmup > 0 else 1.0
    x = step / max(1, total) if per_step else (step // steps_per_epoch) * steps_per_epoch / max(1, total)
    return lr * w * 0.5 * (1.0 + math.cos(math.pi * x))


def train(net, X, T, epochs=10, batch=8, lr=1e-3, seed=0, clip=0.0, warmup=0, per_step=False, log=None):
    """Adam on the mean squared error (gradient clipped to global L2 norm clip
    if clip > 0, learning rate from lr_at); returns the per-epoch mean losses, the
    achieved training rate (TFLOP/s of the MFMA convolutions) and the wall time."""
    import torch
    n = X.shape[0]
    net.set_grad_clip(clip)
    rng = np.random.default_rng(seed)
    f_fwd, f_bwd = net.flops()
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    per_epoch = n // batch
    total = per_epoch * epochs
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(perm[b0:b0 + batch], device=X.device)
            loss = net.train_step(X.index_select(0, idx), T.index_select(0, idx),
                                  lr_at(steps, total, lr, warmup, per_step, per_epoch))
            tot += loss
            cnt += 1
            steps += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"[train] epoch {ep + 1}/{epochs} loss {losses[-1]:.4e}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tflops = steps * batch * (f_fwd + f_bwd) / el / 1e12
    return losses, tflops, el


def time_to_target(solver, start, e_target, max_steps):
    """Wall time and steps of one minimisation from a start function to E <= e_target."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start()
    ss.ss_set_energy_target(solver.ctx, e_target)
    res = solver.minimise(grad_tol=0.0, rel_e_tol=0.0, window=0, max_steps=max_steps, graph_steps=16)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


def ab_compare(net, insts, tol=1e-6, sigmas=(3.0,), pin=0.0, ref_rel_e_tol=1e-9, ref_window=100,
               ref_max_steps=50000, max_steps=50000, coarse_tols=(), noise_amp=1e-3, learned_noise_amp=0.0,
               device="cuda:0", log=None):
    """For each instance: a long ansatz-start run gives E_ref (its stalled energy);
    then the ansatz start and the learned start (for each envelope width sigma,
    with the given pin radius) are flowed until E <= E_ref + tol |E_ref|, and
    again for each coarser tolerance in coarse_tols (keys suffixed "~tol").
    The ansatz start carries the instance's seeded noise of amplitude noise_amp,
    the learned start the same noise at amplitude learned_noise_amp.
    Returns per-instance records; the learned start's time includes building the
    input and running the network."""
    import torch
    m0 = insts[0]
    x = torch.empty((1, m0.Ny, m0.Nx, 2), dtype=torch.float32, device=device)
    corr = torch.empty((1, m0.Ny, m0.Nx, 4), dtype=torch.float32, device=device)
    net.forward(x, out=corr, graph=True)  # capture the forward on these buffers once
    recs = []
    for k, m in enumerate(insts):
        s = ss.Solver("abelian_higgs", m.Nx, m.Ny, m.h, m.params, dtype="f32", device=device)
        s.init_vortices(m.centres, seed=m.seed, noise_amp=noise_amp)
        ref = s.minimise(grad_tol=0.0, rel_e_tol=ref_rel_e_tol, window=ref_window, max_steps=ref_max_steps,
                         graph_steps=16)
        E_ref = ref["energy"]
        target = E_ref + tol * abs(E_ref)

        def ansatz_start():
            s.init_vortices(m.centres, seed=m.seed, noise_amp=noise_amp)

        ta, ra = time_to_target(s, ansatz_start, target, max_steps)
        ansatz_start()
        rec = {"kappa": m.kappa, "n_vortices": len(m.centres), "E_ref": E_ref, "ref_steps": ref["step"],
               "ansatz_s": ta, "ansatz_steps": ra["step"], "ansatz_reached": ra["reason"] == "target",
               "ansatz_E": ra["energy"], "ansatz_E0": s.energy_grad(want_grad=False)[0]}
        for ct in coarse_tols:
            tc, rc = time_to_target(s, ansatz_start, E_ref + ct * abs(E_ref), max_steps)
            rec.update({f"ansatz_s~{ct:g}": tc, f"ansatz_steps~{ct:g}": rc["step"],
                        f"ansatz_reached~{ct:g}": rc["reason"] == "target"})
        for sg in sigmas:
            def learned_start():
                ss.ss_learned_input(s.ctx, m.centres, m.kappa, x.data_ptr())
                net.forward(x, out=corr, graph=True)
                ss.ss_init_learned(s.ctx, m.centres, None, corr.data_ptr(), sigma=sg, pin=pin, seed=m.seed,
                                   noise_amp=learned_noise_amp)

            tl, rl = time_to_target(s, learned_start, target, max_steps)
            learned_start()
            rec.update({f"learned_s@{sg}": tl, f"learned_steps@{sg}": rl["step"],
                        f"learned_reached@{sg}": rl["reason"] == "target", f"learned_E@{sg}": rl["energy"],
                        f"learned_E0@{sg}": s.energy_grad(want_grad=False)[0]})
            for ct in coarse_tols:
                tc, rc = time_to_target(s, learned_start, E_ref + ct * abs(E_ref), max_steps)
                rec.update({f"learned_s@{sg}~{ct:g}": tc, f"learned_steps@{sg}~{ct:g}": rc["step"],
                            f"learned_reached@{sg}~{ct:g}": rc["reason"] == "target"})
        recs.append(rec)
        s.close()
        if log and (k + 1) % 8 == 0:
            log(f"[ab] {k + 1}/{len(insts)}")
    return recs


def summarise(recs, sigma, tol=None, coarse=None):
    """Median time and step ratios (learned / ansatz) over the instances both starts
    brought to the target, the win fraction, and the misses of the learned start;
    for a coarse tolerance of ab_compare when coarse is given."""
    sfx = "" if coarse is None else f"~{coarse:g}"
    key = f"@{sigma}" + sfx
    both = [r for r in recs if r["ansatz_reached" + sfx] and r["learned_reached" + key]]
    ratio = [r["learned_s" + key] / r["ansatz_s" + sfx] for r in both]
    sratio = [r["learned_steps" + key] / max(1, r["ansatz_steps" + sfx]) for r in both]
    return {"sigma": sigma, "tol": coarse if coarse is not None else tol, "instances": len(recs),
            "both_reached": len(both),
            "learned_missed": sum(1 for r in recs if not r["learned_reached" + key]),
            "ansatz_missed": sum(1 for r in recs if not r["ansatz_reached" + sfx]),
            "median_time_ratio": float(np.median(ratio)) if ratio else None,
            "median_step_ratio": float(np.median(sratio)) if sratio else None,
            "learned_win_fraction": float(np.mean([x < 1 for x in ratio])) if ratio else None,
            "median_ansatz_steps": float(np.median([r["ansatz_steps" + sfx] for r in both])) if both else None,
            "median_ansatz_s": float(np.median([r["ansatz_s" + sfx] for r in both])) if both else None,
            "median_learned_s": float(np.median([r["learned_s" + key] for r in both])) if both else None,
            "total_ansatz_s": float(sum(r["ansatz_s" + sfx] for r in recs)),
            "total_learned_s": float(sum(r["learned_s" + key] for r in recs))}


def run_pipeline(n_train=2048, n_test=64, side=256, levels=4, base=32, epochs=20, batch=8, lr=1e-3, seed=0,
                 tol=1e-6, sigmas=(0.0, 3.0), target_steps=150, pin=0.0, coarse_tols=(), clip=0.0,
                 learned_noise_amp=0.0, warmup=0, per_step=False, test_offset=0, save_weights=None,
                 load_weights=None, device="cuda:0", log=print):
    """Data -> training -> A/B on held-out instances test_offset .. test_offset +
    n_test - 1; returns a summary dict. With load_weights the data and training
    steps are skipped and the stored network is evaluated; save_weights stores the
    trained network (flat fp32, exchange order, .npy)."""
    import torch
    t0 = time.perf_counter()
    test_insts = [learned_instance(test_offset + j, 6_000_000, side) for j in range(n_test)]
    net = ss.Net(levels=levels, base=base, cin=2, cout=4, N=batch, H=side, W=side, device=device)
    losses, tflops, t_train, t_data, steps, zero_mse = [], 0.0, 0.0, 0.0, [0], 0.0
    if load_weights:
        net.set_weights(np.load(load_weights).astype(np.float32))
    else:
        train_insts = [learned_instance(i, 5_000_000, side) for i in range(n_train)]
        X, T, steps = generate_dataset(train_insts, batch=64, max_steps=target_steps, device=device, log=log)
        t_data = time.perf_counter() - t0
        zero_mse = float(T.pow(2).mean().item())
        if log:
            log(f"[data] target mean square {zero_mse:.4e} (the loss of predicting no correction)")
        net.set_weights(init_weights(seed, levels, base, 2, 4))
        losses, tflops, t_train = train(net, X, T, epochs=epochs, batch=batch, lr=lr, seed=seed, clip=clip,
                                        warmup=warmup, per_step=per_step, log=log)
        if save_weights:
            np.save(save_weights, net.get_weights())
        del X, T
        torch.cuda.empty_cache()
    # network time of one learned start (batch of one image), after a warm-up
    x1 = torch.zeros((1, side, side, 2), dtype=torch.float32, device=device)  # the time does not depend on values
    o1 = torch.empty((1, side, side, 4), dtype=torch.float32, device=device)
    net.forward(x1, out=o1, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        net.forward(x1, out=o1, graph=True)
    torch.cuda.synchronize()
    infer_ms = (time.perf_counter() - t1) / 20 * 1e3
    if log:
        log(f"[infer] {infer_ms:.3f} ms per image at batch 1")
    recs = ab_compare(net, test_insts, tol=tol, sigmas=sigmas, pin=pin, coarse_tols=coarse_tols,
                      learned_noise_amp=learned_noise_amp, device=device, log=log)
    out = {"summary": [summarise(recs, sg, tol=tol) for sg in sigmas] +
           [summarise(recs, sg, coarse=ct) for ct in coarse_tols for sg in sigmas]}
    out.update({"n_train": n_train, "n_test": n_test, "side": side, "levels": levels, "base": base,
                "epochs": epochs, "batch": batch, "lr": lr, "data_s": t_data,
                "data_median_steps": float(np.median(steps)), "train_s": t_train, "train_TFLOPs": tflops,
                "loss_first_epoch": losses[0] if losses else None, "loss_last_epoch": losses[-1] if losses else None,
                "losses": losses, "tol": tol,
                "target_steps": target_steps, "target_mean_square": zero_mse, "pin": pin, "clip": clip,
                "learned_noise_amp": learned_noise_amp, "warmup": warmup, "per_step": per_step,
                "test_offset": test_offset, "inference_ms_batch1": infer_ms,
                "records": recs})
    net.close()
    return out


def merge_runs(paths, out=None):
    """Summaries over the records of several runs of the same network (held-out
    chunks): the per-instance records are concatenated and summarised again."""
    import json
    runs = [json.load(open(p)) for p in paths]
    recs = [r for run in runs for r in run["records"]]
    first = runs[0]
    sigmas = sorted({s["sigma"] for s in first["summary"]})
    coarse = sorted({s["tol"] for s in first["summary"] if s["tol"] != first["tol"]}, reverse=True)
    res = {"summary": [summarise(recs, sg, tol=first["tol"]) for sg in sigmas] +
           [summarise(recs, sg, coarse=ct) for ct in coarse for sg in sigmas],
           "n_test": len(recs), "parts": [p for p in paths],
           "train": {k: first.get(k) for k in ("n_train", "epochs", "lr", "warmup", "per_step", "clip",
                                               "loss_last_epoch", "losses", "train_s", "train_TFLOPs",
                                               "target_mean_square", "data_s")},
           "inference_ms_batch1": first.get("inference_ms_batch1")}
    print(json.dumps({k: v for k, v in res.items() if k != "train"}), flush=True)
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned initialiser: generate minima, train, compare starts")
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--n-test", type=int, default=64)
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=32)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--target-steps", type=int, default=150, help="flow steps behind each training target")
    ap.add_argument("--pin", type=float, default=0.5, help="radius that pins the zeros of psi at the centres")
    ap.add_argument("--sigmas", default="3", help="envelope widths of the learned start (comma list)")
    ap.add_argument("--clip", type=float, default=0.0, help="global L2 gradient clipping norm (0: off)")
    ap.add_argument("--learned-noise", type=float, default=0.0,
                    help="amplitude of the instance's seeded noise added to the learned start (the ansatz start has 1e-3)")
    ap.add_argument("--coarse-tols", default="1e-3,1e-4",
                    help="coarser relative energy tolerances also timed (comma list, may be empty)")
    ap.add_argument("--warmup", type=int, default=0, help="linear learning-rate warm-up steps")
    ap.add_argument("--per-step-cosine", action="store_true", help="cosine decay per step (default: per epoch)")
    ap.add_argument("--test-offset", type=int, default=0, help="first held-out instance")
    ap.add_argument("--save-weights", default=None, help="store the trained network here (.npy)")
    ap.add_argument("--load-weights", default=None, help="evaluate this stored network (no data, no training)")
    ap.add_argument("--merge", nargs="+", default=None,
                    help="summarise the records of several --out files (held-out chunks) and exit")
    ap.add_argument("--out", default=None, help="write the summary JSON here")
    a = ap.parse_args(argv)
    if a.merge:
        return merge_runs(a.merge, a.out)
    sig = tuple(float(v) for v in a.sigmas.split(","))
    coarse = tuple(float(v) for v in a.coarse_tols.split(",") if v.strip())
    res = run_pipeline(a.n_train, a.n_test, a.side, a.levels, a.base, a.epochs, a.batch, a.lr, sigmas=sig,
                       target_steps=a.target_steps, pin=a.pin, coarse_tols=coarse, clip=a.clip,
                       learned_noise_amp=a.learned_noise, warmup=a.warmup, per_step=a.per_step_cosine,
                       test_offset=a.test_offset, save_weights=a.save_weights, load_weights=a.load_weights,
                       log=lambda m: print(m, flush=True))
    brief = {k: v for k, v in res.items() if k not in ("records", "losses")}
    print(json.dumps(brief), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
