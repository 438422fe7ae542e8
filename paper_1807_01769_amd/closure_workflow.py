"""Learned-closure workflow on one GPU: forced DNS -> filtered samples ->
network training -> coarse LES compared with the filtered DNS.

Every numerical step runs in libfs kernels (fs.Plan, fs.Closure, fs.Mlp,
fs.Les); torch only holds device memory, shuffles sample indices and
averages the FP64 spectra the library returns.

Workflow (all times in the solver's time units):
  1. spin-up: forced DNS from the seeded solenoidal field until the energy
     and the dissipation 2 nu Z are stationary;
  2. collection: every `every` time units the DNS state is cut off to the
     coarse grid's kept cube (|m_a| <= floor((nc-1)/3)); its velocity
     gradients are the features and the subgrid stress the targets;
  3. training: Adam on minibatches of standardised samples (features by one
     RMS over the 9 gradients, targets by per-component RMS), the last
     snapshots held out for validation;
  4. evaluation: from a later held-out DNS snapshot, the DNS, the LES with
     the network and the no-model LES run side by side; their shell spectra
     up to the cutoff are averaged over the window and compared.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import asdict, dataclass

import numpy as np
import torch

from . import fs
from . import inputs


@dataclass
class Config:
    nf: int = 512            # DNS grid
    nc: int = 64             # LES grid
    nu: float = 2e-4
    dt: float = 1e-3         # DNS step
    les_dt_factor: int = 8   # LES step = factor * DNS step
    power: float = 5e-3      # constant injected power
    kf_min: float = 2.0
    kf_max: float = 3.0
    seed: int = 1
    energy0: float = 1.0
    spinup: float = 20.0     # time units of DNS before sampling
    report: float = 0.5      # spin-up progress interval
    nsnap: int = 24          # snapshots collected
    every: float = 0.1       # time between snapshots
    nval: int = 4            # last snapshots kept for validation
    gap: float = 1.0         # DNS time between the last snapshot and the evaluation start
    eval_time: float = 4.0   # evaluation window
    eval_every: float = 0.2  # spectra sampling interval in the window
    iters: int = 6000
    batch: int = 8192
    lr: float = 1e-3
    lr_final: float = 1e-4
    clip: float = 6.0        # clip of the standardised network output
    net_seed: int = 7
    filter: str = "sharp"    # "sharp" cube cutoff or "box" (top-hat, then the cutoff);
                             # several, comma-separated ("sharp,box"), share one DNS run


def _steps(t: float, dt: float) -> int:
    k = int(round(t / dt))
    if abs(k * dt - t) > 1e-9 * max(1.0, t):
        raise ValueError(f"time {t} is not a multiple of the step {dt}")
    return k


def _log(msg: str) -> None:
    print(msg, flush=True)


def _diag(plan: fs.Plan, u: torch.Tensor, nu: float):
    spec, e, z = plan.energy_spectrum(u)
    return spec, float(e.item()), 2.0 * nu * float(z.item())


def spin_up(cfg: Config, plan: fs.Plan, u: torch.Tensor) -> list:
    """Advance the DNS by cfg.spinup; returns the (t, E, eps) history."""
    hist = []
    chunk = _steps(cfg.report, cfg.dt)
    nrep = _steps(cfg.spinup, cfg.dt) // chunk
    _, e, eps = _diag(plan, u, cfg.nu)
    hist.append((0.0, e, eps))
    _log(f"spin-up t=0 E={e:.5f} eps={eps:.5f}")
    t0 = time.perf_counter()
    for r in range(1, nrep + 1):
        plan.step(u, chunk)
        _, e, eps = _diag(plan, u, cfg.nu)
        if not math.isfinite(e):
            raise FloatingPointError("DNS energy is not finite")
        hist.append((r * cfg.report, e, eps))
        _log(f"spin-up t={r * cfg.report:.2f} E={e:.5f} eps={eps:.5f} "
             f"wall={time.perf_counter() - t0:.1f}s")
    return hist


def stationarity(hist: list, window: float) -> dict:
    """Relative drift of E and eps between the two halves of the last window."""
    tend = hist[-1][0]
    last = [h for h in hist if h[0] > tend - window]
    half = len(last) // 2
    if half < 1:
        return {"E_drift": float("nan"), "eps_drift": float("nan")}
    a, b = last[:half], last[half:]
    ea, eb = np.mean([h[1] for h in a]), np.mean([h[1] for h in b])
    da, db = np.mean([h[2] for h in a]), np.mean([h[2] for h in b])
    return {"E_drift": float(abs(eb / ea - 1)), "eps_drift": float(abs(db / da - 1)),
            "E": float(eb), "eps": float(db)}


def collect(cfg: Config, plan: fs.Plan, closures: list, u: torch.Tensor):
    """cfg.nsnap snapshots every cfg.every, filtered by every closure: per
    closure, lists of A [9][P] and tau [6][P]."""
    out = [([], []) for _ in closures]
    k = _steps(cfg.every, cfg.dt)
    for s in range(cfg.nsnap):
        plan.step(u, k)
        for closure, (As, taus) in zip(closures, out):
            _, A, tau = closure.samples(u)
            As.append(A)
            taus.append(tau)
        if s % 4 == 3 or s == cfg.nsnap - 1:
            _log(f"collected {s + 1}/{cfg.nsnap} snapshots")
    return out


def standardise(closure: fs.Closure, As, taus):
    """One RMS over the 9 gradients, per-component RMS of the 6 stresses."""
    m = torch.stack([closure.moments(A, t) for A, t in zip(As, taus)]).mean(0).cpu().numpy()
    a_scale = float(np.sqrt(m[:9].mean()))
    tau_scale = [float(np.sqrt(v)) for v in m[9:]]
    return a_scale, tau_scale


def train(cfg: Config, closure: fs.Closure, As, taus, a_scale, tau_scale):
    xs, ts = [], []
    for A, tau in zip(As, taus):
        x, t = closure.features(A, a_scale, tau, tau_scale)
        xs.append(x)
        ts.append(t)
    ntr = len(xs) - cfg.nval
    xtr, ttr = torch.cat(xs[:ntr]), torch.cat(ts[:ntr])
    xva, tva = torch.cat(xs[ntr:]), torch.cat(ts[ntr:])
    net = fs.Mlp(seed=cfg.net_seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.seed)
    ntrain = xtr.shape[0]
    hist = []
    _, l0 = net.grad(xva, tva)
    _log(f"training on {ntrain} samples, validating on {xva.shape[0]}; "
         f"initial validation loss {float(l0.item()):.4f}")
    t0 = time.perf_counter()
    for it in range(cfg.iters):
        frac = it / max(1, cfg.iters - 1)
        lr = cfg.lr_final + 0.5 * (cfg.lr - cfg.lr_final) * (1 + math.cos(math.pi * frac))
        idx = torch.randint(0, ntrain, (cfg.batch,), device="cuda", generator=g)
        net.train_step(xtr.index_select(0, idx), ttr.index_select(0, idx), lr)
        if (it + 1) % max(1, cfg.iters // 10) == 0:
            _, lv = net.grad(xva, tva)
            _, lt = net.grad(xtr[: xva.shape[0]], ttr[: xva.shape[0]])
            hist.append((it + 1, float(lt.item()), float(lv.item())))
            _log(f"iter {it + 1}: train loss {hist[-1][1]:.4f} val loss {hist[-1][2]:.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # a-priori quality on the validation snapshots: per-component correlation
    y = net.forward(xva)
    corr = []
    for c in range(6):
        a, b = y[:, c].double(), tva[:, c].double()
        a, b = a - a.mean(), b - b.mean()
        corr.append(float((a * b).sum() / torch.sqrt((a * a).sum() * (b * b).sum())))
    return net, {"loss_history": hist, "val_loss0": float(l0.item()), "train_seconds": train_s,
                 "val_correlation": corr}


def _spectrum(plan: fs.Plan, u: torch.Tensor, kc: int) -> np.ndarray:
    spec, _, _ = plan.energy_spectrum(u)
    return spec[: kc + 1].cpu().numpy()


def evaluate(cfg: Config, fine: fs.Plan, coarse: fs.Plan, models: list, u: torch.Tensor):
    """DNS, and per (closure, net, a_scale, tau_scale) in `models` the LES with
    the network and the no-model LES, over cfg.eval_time from the filtered
    state of `u` (advanced in place).  Returns one result per model."""
    kc = (cfg.nc - 1) // 3
    les_dt = cfg.dt * cfg.les_dt_factor
    n_dns = _steps(cfg.eval_every, cfg.dt)
    n_les = _steps(cfg.eval_every, les_dt)
    nwin = int(round(cfg.eval_time / cfg.eval_every))
    cases = []
    for closure, net, a_scale, tau_scale in models:
        uc0, _, _ = closure.samples(u)
        runs = {}
        for name, model in (("model", net), ("no_model", None)):
            runs[name] = {"state": uc0.clone(),
                          "les": fs.Les(coarse, model, a_scale, tau_scale, cfg.clip),
                          "spectra": [], "energy": [], "seconds": 0.0, "finite": True}
        cases.append({"closure": closure, "runs": runs, "dns_spectra": [], "dns_energy": []})
    dns_seconds = 0.0
    for w in range(nwin):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fine.step(u, n_dns)
        torch.cuda.synchronize()
        dns_seconds += time.perf_counter() - t0
        for case in cases:
            uc, _, _ = case["closure"].samples(u)
            s = _spectrum(coarse, uc, kc)
            case["dns_spectra"].append(s)
            case["dns_energy"].append(float(s[1:].sum()))
            for name, r in case["runs"].items():
                if not r["finite"]:
                    continue
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r["les"].step(r["state"], n_les)
                torch.cuda.synchronize()
                r["seconds"] += time.perf_counter() - t0
                sp = _spectrum(coarse, r["state"], kc)
                if not np.all(np.isfinite(sp)):
                    r["finite"] = False
                    _log(f"LES {name} ({case['closure'].filter}) became non-finite at window {w + 1}")
                    continue
                r["spectra"].append(sp)
                r["energy"].append(float(sp[1:].sum()))
            _log(f"eval t={(w + 1) * cfg.eval_every:.2f} {case['closure'].filter}: "
                 f"E_fDNS={case['dns_energy'][-1]:.5f} " +
                 " ".join(f"E_{k}={r['energy'][-1]:.5f}" for k, r in case["runs"].items()
                          if r["energy"]))
    results = []
    for case in cases:
        ref = np.mean(case["dns_spectra"], axis=0)
        out = {"filter": case["closure"].filter, "k": list(range(1, kc + 1)),
               "E_fdns": ref[1:].tolist(), "dns_seconds_per_time": dns_seconds / cfg.eval_time}
        for name, r in case["runs"].items():
            if r["finite"] and len(r["spectra"]) == nwin:
                m = np.mean(r["spectra"], axis=0)
                ratio = m[1:] / ref[1:]
                out[name] = {"E": m[1:].tolist(), "max_rel_err": float(np.abs(ratio - 1).max()),
                             "ratio": ratio.tolist(),
                             "seconds_per_time": r["seconds"] / cfg.eval_time,
                             "ms_per_step": 1e3 * r["seconds"] / (nwin * n_les),
                             "energy_history": r["energy"]}
            else:
                out[name] = {"max_rel_err": float("inf"), "finite": False}
            r["les"].close()
        out["fdns_energy_history"] = case["dns_energy"]
        if "seconds_per_time" in out.get("model", {}):
            out["speedup_model_vs_dns"] = (out["dns_seconds_per_time"] /
                                           out["model"]["seconds_per_time"])
        results.append(out)
    return results


def run(cfg: Config) -> dict:
    """The workflow for every filter in cfg.filter from one DNS run.  With one
    filter, result["training"] and result["evaluation"] are its outcome; with
    several, result["filters"][name] holds each filter's."""
    if not torch.cuda.is_available():
        raise RuntimeError("the closure workflow needs a HIP device")
    filters = [f.strip() for f in cfg.filter.split(",") if f.strip()]
    fine = fs.Plan(cfg.nf, nu=cfg.nu, dt=cfg.dt, forcing_power=cfg.power,
                   forcing_kmin=cfg.kf_min, forcing_kmax=cfg.kf_max)
    coarse = fs.Plan(cfg.nc, nu=cfg.nu, dt=cfg.dt * cfg.les_dt_factor, forcing_power=cfg.power,
                     forcing_kmin=cfg.kf_min, forcing_kmax=cfg.kf_max)
    closures = [fs.Closure(fine, coarse, filter=f) for f in filters]
    u = torch.from_numpy(inputs.random_solenoidal_3d(cfg.nf, seed=cfg.seed, energy=cfg.energy0,
                                                     dtype=np.complex64)).cuda()
    result = {"config": asdict(cfg)}
    hist = spin_up(cfg, fine, u)
    result["spinup"] = {"history": hist, "stationarity": stationarity(hist, min(4.0, cfg.spinup))}
    _log(f"stationarity over the last window: {result['spinup']['stationarity']}")
    samples = collect(cfg, fine, closures, u)
    models, per = [], {}
    for f, closure, (As, taus) in zip(filters, closures, samples):
        a_scale, tau_scale = standardise(closure, As, taus)
        _log(f"filter {f}: training")
        net, tr = train(cfg, closure, As, taus, a_scale, tau_scale)
        per[f] = {"scales": {"a_scale": a_scale, "tau_scale": tau_scale}, "training": tr}
        models.append((closure, net, a_scale, tau_scale))
    del samples
    fine.step(u, _steps(cfg.gap, cfg.dt))
    for f, ev in zip(filters, evaluate(cfg, fine, coarse, models, u)):
        per[f]["evaluation"] = ev
        _log(f"filter {f}: spectral error up to the cutoff: model "
             f"{ev['model'].get('max_rel_err')}, no model {ev['no_model'].get('max_rel_err')}; "
             f"LES {ev['model'].get('ms_per_step')} ms/step; "
             f"speedup vs DNS {ev.get('speedup_model_vs_dns')}")
    if len(filters) == 1:
        result.update(per[filters[0]])
    else:
        result["filters"] = per
    for _, net, _, _ in models:
        net.close()
    for o in (*closures, coarse, fine):
        o.close()
    return result


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    for f, v in asdict(Config()).items():
        ap.add_argument("--" + f.replace("_", "-"), type=type(v), default=v)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    cfg = Config(**{f: getattr(a, f) for f in asdict(Config())})
    res = run(cfg)
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
