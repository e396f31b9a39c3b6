"""Train the learned initial guess of the stage solves on trajectories that the
solver itself generates.

For each trajectory: a seeded Gaussian-random-field initial displacement (zero
velocity) on the deformed cube, stepped by the plain FP64 method (extrapolated
guess, which keeps the ring of past stage solutions).  From the fifth step on,
every step gives one training sample per stage: the four previous stage
solutions H1..H4 and the new one X; the sample is cut into random crops and the
stage's net takes one Adam step on them.  All of it runs in the library's own
kernels (ga_gnet_make_batch, ga_gnet_loss_grad, ga_gnet_adam); by default layer 2's
convolutions run on the BF16 matrix cores, with FP32 master weights (--prec).

The nets start with a zero last layer, i.e. at the plain cubic extrapolation,
and learn the correction.  Output: an .npz with one float32 parameter vector
per stage (``stage0``, ``stage1``, ...) and the run's settings (``meta``, JSON).

    python -m paper_2102_11536_amd.train_gnet --n 128 --p 3 --k 2 \
        --trajectories 500 --steps 16 --out paper_2102_11536_amd/weights/gnet_p3_n128_k2.npz

``--time-gradient N`` only times the loss gradient of one training batch in BF16 and in
FP32 training.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from paper_2102_11536_amd import ga, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "gnet_p3_n128_k2.npz")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def initial_params(seed):
    p = workloads.gnet_random_params(seed)
    p[-(27 * 32 + 1):] = 0.0          # W3, b3 = 0: the net starts at the extrapolation
    return p.astype(np.float32)


def load_weights(path=DEFAULT_WEIGHTS):
    """Per-stage parameter vectors from a file written by this script."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        return [np.asarray(z[f"stage{j}"], dtype=np.float32) for j in range(meta["k"])], meta


def evaluate(pt, k, rho, tau, rtol, mode, nets, nsteps, seed):
    """Mean preconditioned residual of the guess relative to b, and PCG
    iterations, over the solves of one trajectory (steps with a full history)."""
    dev = "cuda:0"
    integ = ga.Integrator(pt, k, rho, tau, rtol=rtol, guess=mode)
    for j, net in enumerate(nets):
        ga.ga_integrator_set_net(integ, j, net)
    U0 = torch.as_tensor(workloads.grf(pt.n_el[0], pt.p, seed=seed), dtype=torch.float64, device=dev)
    state = [torch.zeros(pt.n_free, dtype=torch.float64, device=dev) for _ in range(3 * k)]
    ga.ga_init_state(integ, U0, torch.zeros_like(U0), state)
    ga.ga_step(integ, state, 4)
    ga.ga_solve_stats(pt)
    its = ga.ga_step(integ, state, nsteps)
    st = ga.ga_solve_stats(pt)
    integ.close()
    return {"mean_guess_relres": st["mean_guess_relres"], "fallbacks": st["fallbacks"],
            "mean_iters": float(its.mean())}


def time_gradient(m, S, nb, reps, seed):
    """Mean time of ga_gnet_loss_grad on nb random crops of S^3 on an m^3 grid (inputs
    and targets standard normal, random parameters), in BF16 and in FP32 training:
    {"bf16_ms": .., "fp32_ms": .., ...}."""
    dev = "cuda:0"
    rng = np.random.default_rng(seed)
    T = S - 6
    grid = (m, m, m)
    org = [tuple(int(rng.integers(-3, m - T - 3 + 1)) for _ in range(3)) for _ in range(nb)]
    inp = torch.as_tensor(rng.standard_normal(nb * 4 * S ** 3), dtype=torch.float32, device=dev)
    tgt = torch.as_tensor(rng.standard_normal(nb * T ** 3), dtype=torch.float32, device=dev)
    grad = torch.zeros(ga.GA_GNET_NPARAM, dtype=torch.float32, device=dev)
    out = dict(grid=m, crop=S, batch=nb, reps=reps)
    for name, prec in (("bf16", ga.GA_BF16), ("fp32", ga.GA_FP32)):
        net = ga.GNet(workloads.gnet_random_params(seed))
        ga.ga_gnet_set_train_prec(net, prec)
        for _ in range(2):
            ga.ga_gnet_loss_grad(net, grid, org, S, inp, tgt, grad, want_loss=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ga.ga_gnet_loss_grad(net, grid, org, S, inp, tgt, grad, want_loss=False)
        torch.cuda.synchronize()
        out[f"{name}_ms"] = 1e3 * (time.perf_counter() - t0) / reps
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--rho", type=float, default=0.5)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--trajectories", type=int, default=500)
    ap.add_argument("--steps", type=int, default=16, help="steps per trajectory (samples from step 5 on)")
    ap.add_argument("--crop", type=int, default=30, help="crop edge S (targets (S-6)^3)")
    ap.add_argument("--batch", type=int, default=16, help="crops per sample")
    ap.add_argument("--lr", type=float, default=1e-5)
    ap.add_argument("--lr-min", type=float, default=2e-7)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--eval-steps", type=int, default=24)
    ap.add_argument("--prec", choices=("bf16", "fp32"), default="bf16",
                    help="training arithmetic: layer 2 on BF16 matrix cores, or FP32 throughout")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--time-gradient", type=int, default=0, metavar="N",
                    help="only time N loss gradients of one batch of random crops on the grid of "
                         "free coefficients, in BF16 and in FP32, print one JSON line and exit")
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "training runs on the GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ga.load_library()
    n, p, k = args.n, args.p, args.k
    if args.time_gradient > 0:
        out = time_gradient(n + p - 2, args.crop, args.batch, args.time_gradient, args.seed)
        log(f"[train] gradient: BF16 {out['bf16_ms']:.3f} ms, FP32 {out['fp32_ms']:.3f} ms")
        print(json.dumps(out), flush=True)
        return
    pt = ga.ga_setup_patch(3, n, p, workloads.deformed_cube_ctrl(n, p))
    lam = ga.ga_lambda_max(pt, 25)
    tau = 0.5 * math.sqrt(ga.ga_stability_limit(args.rho) / lam)
    log(f"[train] n={n} p={p} k={k} n_free={pt.n_free} tau={tau:.4e} trajectories={args.trajectories}")
    nets = [ga.GNet(initial_params(args.seed + j)) for j in range(k)]
    for net in nets:
        ga.ga_gnet_set_train_prec(net, ga.GA_BF16 if args.prec == "bf16" else ga.GA_FP32)
    S, nb, T = args.crop, args.batch, args.crop - 6
    if min(pt.mf) < T:
        raise SystemExit("grid smaller than the crop target")
    f32 = dict(dtype=torch.float32, device=dev)
    inp = torch.zeros(nb * 4 * S ** 3, **f32)
    tgt = torch.zeros(nb * T ** 3, **f32)
    grad = torch.zeros(ga.GA_GNET_NPARAM, **f32)
    H = [[torch.zeros(pt.n_free, dtype=torch.float64, device=dev) for _ in range(4)] for _ in range(k)]
    X = [torch.zeros(pt.n_free, dtype=torch.float64, device=dev) for _ in range(k)]
    rng = np.random.default_rng(args.seed)
    total = args.trajectories * max(0, args.steps - 4)
    done = 0
    hist_ratio = [[] for _ in range(k)]
    hist_base = [[] for _ in range(k)]
    t0 = time.time()
    for tr in range(args.trajectories):
        integ = ga.Integrator(pt, k, args.rho, tau, rtol=args.rtol, guess=ga.GA_GUESS_EXTRAP)
        U0 = torch.as_tensor(workloads.grf(n, p, seed=10_000 + tr), dtype=torch.float64, device=dev)
        state = [torch.zeros(pt.n_free, dtype=torch.float64, device=dev) for _ in range(3 * k)]
        ga.ga_init_state(integ, U0, torch.zeros_like(U0), state)
        for step in range(args.steps):
            sample = step >= 4
            if sample:
                for j in range(k):
                    for a in range(4):
                        ga.ga_stage_solution(integ, j, a, H[j][a])
            ga.ga_step(integ, state, 1, record_iters=False)
            if not sample:
                continue
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1 + math.cos(math.pi * done / max(1, total)))
            for j in range(k):
                ga.ga_stage_solution(integ, j, 0, X[j])
                org = [tuple(int(rng.integers(-3, pt.mf[a] - T - 3 + 1)) for a in range(3)) for _ in range(nb)]
                ga.ga_gnet_make_batch(nets[j], pt, H[j], X[j], org, S, inp, tgt)
                loss = ga.ga_gnet_loss_grad(nets[j], pt.mf, org, S, inp, tgt, grad)
                ga.ga_gnet_adam(nets[j], grad, lr)
                base = float(torch.mean(tgt.double() ** 2))   # loss of the plain extrapolation
                hist_ratio[j].append(loss / base if base > 0 else 1.0)
                hist_base[j].append(base)
            done += 1
        integ.close()
        if (tr + 1) % max(1, args.trajectories // 20) == 0 or tr + 1 == args.trajectories:
            recent = [float(np.mean(h[-50:])) if h else float("nan") for h in hist_ratio]
            log(f"[train] trajectory {tr + 1}/{args.trajectories}  {time.time() - t0:.0f}s  "
                f"loss/extrapolation-loss per stage (last 50): " + " ".join(f"{r:.4f}" for r in recent)
                + "  extrapolation loss: " + " ".join(f"{np.mean(b[-50:]):.3e}" for b in hist_base))
    params = [ga.ga_gnet_get_params(net) for net in nets]
    evals = {}
    for name, mode in (("extrapolation", ga.GA_GUESS_EXTRAP), ("learned", ga.GA_GUESS_LEARNED)):
        evals[name] = evaluate(pt, k, args.rho, tau, args.rtol, mode, nets, args.eval_steps, seed=99_999)
        log(f"[train] held-out trajectory, {name} guess: {evals[name]}")
    meta = dict(n=n, p=p, k=k, rho=args.rho, tau=tau, rtol=args.rtol, trajectories=args.trajectories,
                steps=args.steps, crop=S, batch=nb, lr=args.lr, seed=args.seed, prec=args.prec,
                final_ratio=[float(np.mean(h[-200:])) if h else None for h in hist_ratio],
                seconds=time.time() - t0, heldout=evals)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, meta=np.array(json.dumps(meta)), **{f"stage{j}": params[j] for j in range(k)})
    log(f"[train] wrote {args.out}: {json.dumps(meta)}")


if __name__ == "__main__":
    main()
