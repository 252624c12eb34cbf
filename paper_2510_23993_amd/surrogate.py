"""Training and evaluation driver of the learned chemistry surrogate.

All device work runs in libchem's kernels (the implicit integrator makes the
training pairs, chem_surrogate_pairs turns them into features and targets,
the chem_mlp_* kernels standardise, sample, run forward and backward passes
and Adam); this module schedules those calls and reads and writes the
weights file whose format chem_load_surrogate documents.

    python -m paper_2510_23993_amd.surrogate train --out FILE [--pairs N] [--steps S]
    python -m paper_2510_23993_amd.surrogate evaluate --weights FILE [--nz NZ]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "surrogate_m9.bin")
MAGIC = b"CHEMSURR"
NIN, NH, NOUT, NSPEC = 12, 256, 10, 9
SIZES = (NIN, NH, NH, NH, NOUT)


def n_params():
    return sum(a * b + b for a, b in zip(SIZES[:-1], SIZES[1:]))


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), +1/sqrt(fan_in)) for every weight and bias."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        lim = 1.0 / math.sqrt(a)
        out.append(rng.uniform(-lim, lim, a * b))
        out.append(rng.uniform(-lim, lim, b))
    return np.concatenate(out).astype(np.float32)


def write_weights(path, params, mean_x, sd_x, mean_t, sd_t, env_lo, env_hi, mech_hash):
    params = np.asarray(params, dtype="<f4")
    assert params.size == n_params()
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<5i", 1, NIN, NH, NOUT, NSPEC))
        f.write(struct.pack("<Q", mech_hash))
        f.write(params.tobytes())
        for a in (mean_x, sd_x, mean_t, sd_t):
            f.write(np.asarray(a, dtype="<f4").tobytes())
        for a in (env_lo, env_hi):
            f.write(np.asarray(a, dtype="<f8").tobytes())


def read_weights(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError("not a surrogate weights file")
        hdr = struct.unpack("<5i", f.read(20))
        (mech_hash,) = struct.unpack("<Q", f.read(8))
        params = np.frombuffer(f.read(4 * n_params()), dtype="<f4").copy()
        norm = np.frombuffer(f.read(4 * (2 * NIN + 2 * NOUT)), dtype="<f4").copy()
        env = np.frombuffer(f.read(8 * 2 * NIN), dtype="<f8").copy()
    return {"header": hdr, "hash": mech_hash, "params": params,
            "mean_x": norm[:NIN], "sd_x": norm[NIN:2 * NIN], "mean_t": norm[2 * NIN:2 * NIN + NOUT],
            "sd_t": norm[2 * NIN + NOUT:], "env_lo": env[:NIN], "env_hi": env[NIN:]}


def _dt_buckets(dt, nb=32):
    """Quantise per-cell dt to nb log-spaced values (one integration call each)."""
    lo, hi = np.log(dt.min()), np.log(dt.max())
    if hi - lo < 1e-12:
        return np.zeros(dt.size, dtype=np.int64), np.array([dt[0]])
    q = np.clip(np.round((np.log(dt) - lo) / (hi - lo) * (nb - 1)), 0, nb - 1).astype(np.int64)
    vals = np.exp(lo + (hi - lo) * np.arange(nb) / (nb - 1))
    return q, vals


def generate_pairs(ctx, n_states, seed, rtol=1e-9, atol=1e-20, chunk=1 << 20, chain=2, log=print):
    """Training pairs from the GPU integrator: states of the training
    distribution, each advanced `chain` times by its own dt (trajectory
    continuation).  Returns raw float32 device tensors X [N][12], T [N][10]."""
    import torch
    import paper_2510_23993_amd as chem
    from synth import fields
    # the pairs go straight into one buffer; cells the integrator did not
    # finish are dropped by a row gather (the library's take kernel)
    Xall = torch.empty((n_states * chain, NIN), dtype=torch.float32, device="cuda")
    Tall = torch.empty((n_states * chain, NOUT), dtype=torch.float32, device="cuda")
    off = 0
    dropped = 0
    t0 = time.perf_counter()
    for ci, start in enumerate(range(0, n_states, chunk)):
        n = min(chunk, n_states - start)
        c = fields.c5_training_states(n, seed=seed * 1000 + ci)
        q, vals = _dt_buckets(c.dt)
        for bi in np.unique(q):
            idx = np.where(q == bi)[0]
            m = idx.size
            dt = float(vals[bi])
            T = torch.as_tensor(c.T[idx], device="cuda")
            p = torch.as_tensor(c.p[idx], device="cuda")
            Y = torch.as_tensor(np.ascontiguousarray(c.Y[:, idx]), device="cuda")
            rho = torch.empty(m, dtype=torch.float64, device="cuda")
            e = torch.empty_like(rho)
            ctx.prepare_state(T, p, Y, rho, e)
            dtv = torch.full((m,), dt, dtype=torch.float64, device="cuda")
            status = torch.empty(m, dtype=torch.uint8, device="cuda")
            for _ in range(chain):
                Y1, T1 = Y.clone(), T.clone()
                ctx.integrate(rho, e, Y1, T1, dt, rtol, atol, status=status)
                X, Tg = Xall[off:off + m], Tall[off:off + m]
                ctx.surrogate_pairs(rho, Y, T, Y1, T1, dtv, X, Tg)
                ok = np.flatnonzero(status.cpu().numpy() == chem.ST_DONE)
                if ok.size < m:
                    Xk = torch.empty((ok.size, NIN), dtype=torch.float32, device="cuda")
                    Tk = torch.empty((ok.size, NOUT), dtype=torch.float32, device="cuda")
                    chem.MLP.take(torch.as_tensor(ok, dtype=torch.int64, device="cuda"), X, Tg, Xk, Tk)
                    Xall[off:off + ok.size].copy_(Xk)
                    Tall[off:off + ok.size].copy_(Tk)
                dropped += m - ok.size
                off += ok.size
                Y, T = Y1, T1
        log(f"pairs: chunk {ci} done, {off} pairs, {time.perf_counter() - t0:.1f} s")
    return Xall[:off], Tall[:off], dropped


def save_checkpoint(path, p, m, v, step, steps, batch, seed):
    """Optimiser state after `step` steps (parameters, Adam moments) and the
    run's schedule, as an .npz of plain arrays."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=p.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
             schedule=np.array([step, steps, batch, seed], dtype=np.int64))
    os.replace(tmp, path)


def train(X, Tg, steps=20000, batch=4096, seed=7, lr0=1e-3, lr1=1e-5, val_frac=0.02, log=print,
          checkpoint=None, checkpoint_every=0, resume=None, stop_after=None):
    """Standardises the pairs in place, trains with Adam and a cosine
    learning-rate decay, and returns (params, normalisation, history).

    checkpoint: path of an .npz the optimiser state is written to every
    `checkpoint_every` steps (0: only at the end or at `stop_after`).
    resume: such a file; training continues after its step with the same
    schedule (the minibatches are a function of (seed, step), so a resumed
    run reproduces an uninterrupted one bit for bit, given the same pairs).
    stop_after: end after this step (the state is checkpointed)."""
    import torch
    import paper_2510_23993_amd as chem
    M = chem.MLP
    N = X.shape[0]
    acc = torch.zeros(2 * NIN, dtype=torch.float64, device="cuda")
    mean_x, sd_x = (torch.zeros(NIN, dtype=torch.float32, device="cuda") for _ in range(2))
    mean_t, sd_t = (torch.zeros(NOUT, dtype=torch.float32, device="cuda") for _ in range(2))
    lo, hi = (torch.zeros(NIN, dtype=torch.float64, device="cuda") for _ in range(2))
    scratch = torch.zeros(2 * NIN, dtype=torch.int32, device="cuda")
    M.colrange(X, scratch, lo, hi)
    M.colstats(X, acc, mean_x, sd_x)
    M.colstats(Tg, acc, mean_t, sd_t)
    M.standardize(X, mean_x, sd_x)
    M.standardize(Tg, mean_t, sd_t)
    n_val = max(batch, int(val_frac * N))
    n_tr = N - n_val
    # held-out rows: a seeded permutation (the pairs arrive grouped by dt);
    # the training rows keep their order.  Rows are gathered by the
    # library's take kernel.
    perm = np.random.default_rng(seed).permutation(N)
    va = torch.as_tensor(perm[n_tr:], dtype=torch.int64, device="cuda")
    tr = torch.as_tensor(np.sort(perm[:n_tr]), dtype=torch.int64, device="cuda")
    Xva = torch.empty((n_val, NIN), dtype=torch.float32, device="cuda")
    Tva = torch.empty((n_val, NOUT), dtype=torch.float32, device="cuda")
    Xtr = torch.empty((n_tr, NIN), dtype=torch.float32, device="cuda")
    Ttr = torch.empty((n_tr, NOUT), dtype=torch.float32, device="cuda")
    M.take(va, X, Tg, Xva, Tva)
    M.take(tr, X, Tg, Xtr, Ttr)
    p = torch.as_tensor(init_params(seed), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
    first = 1
    if resume is not None:
        with np.load(resume, allow_pickle=False) as ck:
            done, c_steps, c_batch, c_seed = (int(x) for x in ck["schedule"])
            if (c_steps, c_batch, c_seed) != (steps, batch, seed):
                raise ValueError(f"checkpoint schedule {(c_steps, c_batch, c_seed)} differs from "
                                 f"{(steps, batch, seed)}")
            p.copy_(torch.as_tensor(ck["params"]))
            m.copy_(torch.as_tensor(ck["m"]))
            v.copy_(torch.as_tensor(ck["v"]))
        first = done + 1
        log(f"resumed after step {done}")
    last = steps if stop_after is None else min(steps, stop_after)
    Xb = torch.empty((batch, NIN), dtype=torch.float32, device="cuda")
    Tb = torch.empty((batch, NOUT), dtype=torch.float32, device="cuda")
    out = torch.empty((batch, NOUT), dtype=torch.float32, device="cuda")
    dout = torch.empty_like(out)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = M.workspace(batch)

    def val_loss():
        tot, k = 0.0, 0
        for s in range(0, n_val - batch + 1, batch):
            M.forward(p, Xva[s:s + batch], out, ws, mode=0)
            M.mse(out, Tva[s:s + batch], dout, loss)
            tot += float(loss.item())
            k += 1
        return tot / max(k, 1)

    hist = []
    t0 = time.perf_counter()
    for step in range(first, last + 1):
        lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * (step - 1) / steps))
        M.gather(Xtr, Ttr, batch, seed, step, Xb, Tb)
        M.forward(p, Xb, out, ws, mode=0)
        M.mse(out, Tb, dout, loss)
        M.backward(p, Xb, ws, dout, g)
        M.adam(p, g, m, v, step, lr)
        if step == 1 or step % 2000 == 0 or step == last:
            tl = float(loss.item())
            hist.append({"step": step, "train_loss": tl, "lr": lr, "s": time.perf_counter() - t0})
            log(f"step {step}: train loss {tl:.3e}, lr {lr:.2e}, {time.perf_counter() - t0:.1f} s")
        if checkpoint and (step == last or (checkpoint_every and step % checkpoint_every == 0)):
            save_checkpoint(checkpoint, p, m, v, step, steps, batch, seed)
    hist.append({"step": last, "val_loss": val_loss()})
    log(f"validation loss {hist[-1]['val_loss']:.3e}")
    span = hi - lo
    norm = {"mean_x": mean_x.cpu().numpy(), "sd_x": sd_x.cpu().numpy(), "mean_t": mean_t.cpu().numpy(),
            "sd_t": sd_t.cpu().numpy(), "env_lo": (lo - 0.02 * span).cpu().numpy(),
            "env_hi": (hi + 0.02 * span).cpu().numpy()}
    return p.cpu().numpy(), norm, hist


def evaluate(weights, nz=128, rtol=1e-8, atol=1e-14, surr_rtols=(1e-5,), log=print):
    """Detonation-patch field 256 x 256 x nz (seed 1005) integrated without
    and with the surrogate pass (one run per trust tolerance); best of three
    device times, fallback rate, rejection reasons and statistics."""
    import torch
    import paper_2510_23993_amd as chem
    from synth import fields
    mech = chem.Mechanism(fields.M9_PATH)
    cells = fields.c2_field(256, 256, nz, seed=1005)
    n = cells.T.size
    T0 = torch.as_tensor(cells.T, device="cuda")
    p = torch.as_tensor(cells.p, device="cuda")
    Y0 = torch.as_tensor(cells.Y, device="cuda").contiguous()
    res = {"cells": n, "runs": []}
    for surr in [None] + list(surr_rtols):
        ctx = chem.Context(mech)
        if surr is not None:
            ctx.load_surrogate(weights)
            ctx.set_option("surrogate", 1)
            ctx.set_option("surr_rtol", surr)
        rho = torch.empty(n, dtype=torch.float64, device="cuda")
        e = torch.empty_like(rho)
        ctx.prepare_state(T0, p, Y0, rho, e)
        Y, T = torch.empty_like(Y0), torch.empty_like(T0)
        status = torch.empty(n, dtype=torch.uint8, device="cuda")
        best = None
        for _ in range(3):
            Y.copy_(Y0)
            T.copy_(T0)
            st = ctx.integrate(rho, e, Y, T, cells.dt, rtol, atol, status=status)
            if best is None or st["t_total_ms"] < best["t_total_ms"]:
                best = st
        best["status_counts"] = np.bincount(status.cpu().numpy(), minlength=8).tolist()
        best["surr_rtol"] = surr
        if surr is not None:
            best["fallback_rate"] = best["n_fallback"] / max(1, best["n_fallback"] + best["n_surrogate"])
            best["speedup"] = res["runs"][0]["t_total_ms"] / best["t_total_ms"]
        res["runs"].append(best)
        log(f"surr_rtol {surr}: {best['t_total_ms']:.2f} ms, status {best['status_counts']}, "
            f"rejections {best['surr_reject']}")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--pairs", type=int, default=10_000_000)
    t.add_argument("--steps", type=int, default=20000)
    t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--seed", type=int, default=1005)
    t.add_argument("--report", default=None)
    t.add_argument("--checkpoint", default=None, help="optimiser-state file (.npz), written at the end")
    t.add_argument("--checkpoint-every", type=int, default=0, help="also every this many steps")
    t.add_argument("--resume", default=None, help="continue from this optimiser-state file")
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ev.add_argument("--nz", type=int, default=128)
    ev.add_argument("--surr-rtol", type=float, nargs="+", default=[1e-5])
    a = ap.parse_args(argv)
    sys.path.insert(0, ROOT)
    import torch
    import paper_2510_23993_amd as chem
    from synth import fields
    torch.cuda.set_device(0)
    log = lambda s: print(s, flush=True)   # noqa: E731
    if a.cmd == "train":
        mech = chem.Mechanism(fields.M9_PATH)
        ctx = chem.Context(mech)
        t0 = time.perf_counter()
        X, Tg, dropped = generate_pairs(ctx, a.pairs // 2, a.seed, log=log)
        t_gen = time.perf_counter() - t0
        log(f"{X.shape[0]} pairs ({dropped} dropped) in {t_gen:.1f} s")
        params, norm, hist = train(X, Tg, steps=a.steps, batch=a.batch, seed=a.seed, log=log,
                                   checkpoint=a.checkpoint, checkpoint_every=a.checkpoint_every,
                                   resume=a.resume)
        write_weights(a.out, params, norm["mean_x"], norm["sd_x"], norm["mean_t"], norm["sd_t"],
                      norm["env_lo"], norm["env_hi"], mech.hash)
        log(f"wrote {a.out}")
        if a.report:
            with open(a.report, "w") as f:
                json.dump({"pairs": int(X.shape[0]), "dropped": dropped, "t_generate_s": t_gen,
                           "history": hist}, f, indent=1)
    else:
        print(json.dumps(evaluate(a.weights, nz=a.nz, surr_rtols=a.surr_rtol, log=log)))


if __name__ == "__main__":
    main()
