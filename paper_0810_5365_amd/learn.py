"""Learned preconditioner: training data, training loop and the solve comparison.

Training data (per gauge field, generated on the fly on the GPU):
  * Gaussian sources psi;
  * near-null vectors from the plain solver: a few loose inverse iterations
    v <- (M^dag M)^-1 v with the library's CG, which amplify the low modes of M;
    training vectors are random complex combinations of them.
For each psi the pair (M psi, psi) is formed with the library's FP32 Wilson
operator, and the network N is trained so that N(M psi) ~ psi:
    loss = mean over the batch of ||N(M psi) - psi||^2 / ||psi||^2,
with Adam on float32 master weights (cosine-decayed learning rate); the kernels
may run the weights at 16 bits.  The flexible GMRES uses the even-even block of
N as its preconditioner for the Schur complement Mhat, since (M^-1)_ee = Mhat^-1.

Solve comparison on unseen fields: the plain solver (even-odd CG on
Mhat^dag Mhat with FP32 storage and FP64 reliable updates), flexible GMRES
without the network, and flexible GMRES with the trained network (FP32 cycles,
16-bit weights), all to ||b - M x|| / ||b|| <= tol recomputed in float64.
Everything numeric runs in the library's HIP kernels; this module only
marshals tensors and drives the loop.
"""
import ctypes
import time

import numpy as np
import torch

import lattice_synth as ls

from . import wdirac as w
from . import ptconv as pt

BC = (1, 1, 1, -1)


class Field:
    """One gauge field on the device, with its lattice."""

    def __init__(self, ctx, dims, eps, seed, recon=12):
        self.ctx, self.dims, self.seed = ctx, tuple(dims), seed
        self.g = w.Gauge(ctx, dims, BC, recon)
        self.g.upload(ls.gauge_field(dims, eps, seed))
        self.lat = w.lattice(dims, BC)
        self.V = int(np.prod(dims))

    def close(self):
        self.g.close()


def gaussian_full(field, n, seed, prec=w.F32):
    """n Gaussian FULL spinors, packed at prec (drawn on the host, seeded)."""
    X, Y, Z, T = field.dims
    psi = ls.gaussian_complex((n, T, Z, Y, X, 4, 3), seed, ls.STREAM_SPINOR)
    return w.pack(field.ctx, field.lat, w.FULL, prec, psi, n)


def near_null_vectors(field, kappa, n, seed, iters=3, tol=1e-2, maxiter=40):
    """n near-null vectors (FP32 FULL packed): loose inverse iteration with the plain CG on M^dag M."""
    ctx, lat = field.ctx, field.lat
    v = gaussian_full(field, n, seed, w.F64)
    hb64 = w.spinor_bytes(lat, w.FULL, w.F64)
    x = torch.zeros_like(v)
    prm = w.solver_params(tol=tol, maxiter=maxiter, sloppy=w.F32)
    info = w.WdSolverInfo()
    nrm = (ctypes.c_double * 1)()
    for _ in range(iters):
        for k in range(n):
            bk, xk = v.data_ptr() + k * hb64, x.data_ptr() + k * hb64
            w.wd_cg_solve(field.g.handle, kappa, w.FULL, ctypes.byref(prm), bk, xk, ctypes.byref(info),
                          ok=(w.WD_OK, w.WD_ENOCONV))
            w.wd_norm2(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 1, xk, nrm)
            s = 1.0 / np.sqrt(nrm[0])
            # b = x / |x|  (copy, then scale in place: b += (s - 1) b), and reset the guess
            w.wd_spinor_convert(ctx.handle, ctypes.byref(lat), w.FULL, 1, w.F64, xk, w.F64, bk)
            w.wd_caxpy(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 1, s - 1.0, 0.0, bk, bk)
            x[k * hb64:(k + 1) * hb64].zero_()
    out = w.new_field(lat, w.FULL, w.F32, n)
    w.wd_spinor_convert(ctx.handle, ctypes.byref(lat), w.FULL, n, w.F64, v.data_ptr(), w.F32, out.data_ptr())
    return out


def mix_vectors(field, basis, nb, n, gen):
    """n random complex combinations of the nb FP32 FULL vectors in `basis`, normalised to unit mean variance."""
    ctx, lat = field.ctx, field.lat
    hb = w.spinor_bytes(lat, w.FULL, w.F32)
    out = torch.zeros(hb * n, dtype=torch.uint8, device="cuda")
    c = torch.randn((n, nb, 2), generator=gen, dtype=torch.float64)
    scale = np.sqrt(field.V * 12 / nb)       # each basis vector has unit norm
    for i in range(n):
        for k in range(nb):
            w.wd_caxpy(ctx.handle, ctypes.byref(lat), w.FULL, w.F32, 1, float(c[i, k, 0]) * scale,
                       float(c[i, k, 1]) * scale, basis.data_ptr() + k * hb, out.data_ptr() + i * hb)
    return out


def make_pairs(field, kappa, psi, n):
    """(features of M psi, features of psi) for n packed FP32 FULL spinors psi."""
    ctx, lat = field.ctx, field.lat
    mpsi = w.new_field(lat, w.FULL, w.F32, n)
    w.wd_apply_M(field.g.handle, kappa, w.FULL, 0, w.F32, n, psi.data_ptr(), mpsi.data_ptr())
    return pt.spinor_to_features(ctx, lat, mpsi, n), pt.spinor_to_features(ctx, lat, psi, n)


def batch_loss(net, field, x, t, n):
    y = net(x, field.g, n)
    d = (y - t).view(n, -1)
    return ((d * d).sum(1) / (t.view(n, -1) ** 2).sum(1)).mean()


def train(net, fields, kappa, pairs_per_field=512, batch=8, epochs=1, lr=2e-3, n_null=16, seed=0, log=None,
          time_budget_s=None, cosine=True):
    """Train `net` on the given fields; returns a history dict.  cosine: the learning
    rate decays from lr to 0 over the run as 0.5 (1 + cos(pi step / steps))."""
    gen = torch.Generator().manual_seed(seed)
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    total_steps = max(1, epochs * max(1, pairs_per_field // batch) * len(fields))
    sched = torch.optim.lr_scheduler.LambdaLR(
        opt, (lambda k: 0.5 * (1.0 + np.cos(np.pi * min(k, total_steps) / total_steps))) if cosine else (lambda k: 1.0))
    hist = {"loss": [], "seconds": 0.0, "pairs": 0}
    t0 = time.perf_counter()
    nulls = []
    for fi, f in enumerate(fields):
        nulls.append(near_null_vectors(f, kappa, n_null, seed=1000 * (fi + 1) + seed))
    torch.cuda.synchronize()
    hist["near_null_seconds"] = time.perf_counter() - t0
    steps_per_field = max(1, pairs_per_field // batch)
    for ep in range(epochs):
        for s in range(steps_per_field):
            for fi, f in enumerate(fields):
                if s % 2 == 0:
                    psi = gaussian_full(f, batch, seed=10 ** 6 * (ep + 1) + 1000 * s + fi)
                else:
                    psi = mix_vectors(f, nulls[fi], n_null, batch, gen)
                x, t = make_pairs(f, kappa, psi, batch)
                loss = batch_loss(net, f, x, t, batch)
                opt.zero_grad()
                loss.backward()
                opt.step()
                sched.step()
                hist["loss"].append(loss.item())
                hist["pairs"] += batch
            if log and s % 8 == 0:
                log("epoch %d step %d/%d loss %.4f" % (ep, s, steps_per_field, hist["loss"][-1]))
            if time_budget_s and time.perf_counter() - t0 > time_budget_s:
                break
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    return hist


def evaluate_loss(net, fields, kappa, n=8, seed=777):
    out = []
    with torch.no_grad():
        for fi, f in enumerate(fields):
            psi = gaussian_full(f, n, seed + fi)
            x, t = make_pairs(f, kappa, psi, n)
            out.append(float(batch_loss(net, f, x, t, n)))
    return float(np.mean(out))


def solve_compare(net, field, kappa, tol=1e-10, restart=16, seed=4242, maxiter=4000):
    """Plain EO-CG vs flexible GMRES without and with the network on one field."""
    ctx, lat = field.ctx, field.lat
    X, Y, Z, T = field.dims
    b = ls.gaussian_complex((T, Z, Y, X, 4, 3), seed, ls.STREAM_SPINOR)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    res = {}

    def run(name, fn):
        fx = torch.zeros_like(fb)
        info = w.WdSolverInfo()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(fx, info)
        torch.cuda.synchronize()
        d = info.as_dict()
        d["wall_s"] = time.perf_counter() - t0
        res[name] = d
        return fx

    prm = w.solver_params(tol=tol, maxiter=maxiter, sloppy=w.F32, delta=-1.0)   # library default (1e-5)
    run("plain_cg_f32", lambda fx, info: w.wd_wilson_solve(field.g.handle, kappa, ctypes.byref(prm), fb.data_ptr(),
                                                            fx.data_ptr(), ctypes.byref(info)))
    prm_g = w.solver_params(tol=tol, maxiter=maxiter, sloppy=w.F32, delta=-1.0)   # library default (1e-5)
    run("fgmres_no_net", lambda fx, info: w.wd_fgmres_solve(field.g.handle, kappa, ctypes.byref(prm_g), restart, 0,
                                                            None, None, w.F32, fb.data_ptr(), fx.data_ptr(),
                                                            ctypes.byref(info), ok=(w.WD_OK, w.WD_ENOCONV)))
    if net is not None:
        ws = net.storage()
        widths = (ctypes.c_int * len(net.widths))(*net.widths)
        ptrs = (ctypes.c_void_p * len(ws))(*[t.data_ptr() for t in ws])
        xl = run("fgmres_learned", lambda fx, info: w.wd_fgmres_solve(
            field.g.handle, kappa, ctypes.byref(prm_g), restart, len(ws), widths, ptrs, net.wprec, fb.data_ptr(),
            fx.data_ptr(), ctypes.byref(info), ok=(w.WD_OK, w.WD_ENOCONV)))
        res["x_learned"] = xl
    res["b"] = b
    return res


def load_net(path, wprec=w.BF16, device="cuda"):
    """A PTNet with the float32 weights saved by `main(--save ...)`."""
    d = np.load(path)
    widths = tuple(int(c) for c in d["widths"])
    net = pt.PTNet(widths, wprec, device=device)
    with torch.no_grad():
        for k, Wp in enumerate(net.weights):
            Wp.copy_(torch.from_numpy(d["arr_%d" % k]))
    return net


DEFAULT_WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__), "data",
                                             "ptnet_16c32_eps0.7_kappa0.1248.npz")


def main(argv=None):
    """Train on seeded fields and compare solvers on unseen ones; prints one JSON line.

    python -m paper_0810_5365_amd.learn [--dims 16 16 16 32] [--eps 0.7] [--kappa 0.1248]
        [--train-fields 8] [--test-fields 4] [--pairs 512] [--epochs 1] [--wprec bf16] [--save W.npz]
    """
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument("--eps", type=float, default=0.7)
    ap.add_argument("--kappa", type=float, default=0.1248)
    ap.add_argument("--train-fields", type=int, default=8)
    ap.add_argument("--test-fields", type=int, default=4)
    ap.add_argument("--pairs", type=int, default=512, help="training pairs per field")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--n-null", type=int, default=16)
    ap.add_argument("--widths", type=int, nargs="+", default=[4, 8, 8, 4])
    ap.add_argument("--wprec", default="bf16")
    ap.add_argument("--restart", type=int, default=16)
    ap.add_argument("--time-budget", type=float, default=None, help="seconds of training at most")
    ap.add_argument("--no-cosine", action="store_true", help="constant learning rate")
    ap.add_argument("--save", default=None)
    args = ap.parse_args(argv)
    log = lambda m: print("learn: " + m, file=sys.stderr, flush=True)
    ctx = w.Context(0)
    train_f = [Field(ctx, args.dims, args.eps, 5001 + i) for i in range(args.train_fields)]
    net = pt.PTNet(tuple(args.widths), w.PREC_BY_NAME[args.wprec])
    net.init_identity()
    loss0 = evaluate_loss(net, train_f, args.kappa)
    log("initial loss %.4f; training" % loss0)
    hist = train(net, train_f, args.kappa, args.pairs, args.batch, args.epochs, args.lr, args.n_null, log=log,
                 time_budget_s=args.time_budget, cosine=not args.no_cosine)
    for f in train_f:
        f.close()
    if args.save:
        np.savez(args.save, *[p.detach().cpu().numpy() for p in net.weights], widths=np.array(args.widths))
    test_f = [Field(ctx, args.dims, args.eps, 6001 + i) for i in range(args.test_fields)]
    out = {"dims": args.dims, "eps": args.eps, "kappa": args.kappa, "widths": args.widths, "wprec": args.wprec,
           "epochs": args.epochs,
           "train": {"pairs": hist["pairs"], "seconds": round(hist["seconds"], 2),
                     "near_null_seconds": round(hist["near_null_seconds"], 2), "loss_initial": loss0,
                     "loss_final_train": float(np.mean(hist["loss"][-8:]))},
           "test_loss": evaluate_loss(net, test_f, args.kappa), "solves": []}
    for f in test_f:
        r = solve_compare(net, f, args.kappa, restart=args.restart)
        r.pop("x_learned", None)
        r.pop("b", None)
        r["field_seed"] = f.seed
        out["solves"].append(r)
        log("field %d: " % f.seed + ", ".join("%s %d it %.3f s resid %.2e" % (k, v["iters"], v["wall_s"], v["true_resid_M"])
                                              for k, v in r.items() if isinstance(v, dict)))
        f.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
