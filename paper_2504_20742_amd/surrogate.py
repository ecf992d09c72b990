"""Learned surrogate of the stiff phase-change source Q(U, dt).

Builds the training set from the solver itself (exact sub-cycled source of the
GPU library on source-active runs), fits the normalisation and the training
envelope, trains the 17 -> 256 -> 256 -> 15 network with the library's own
MFMA forward/backward and Adam kernels, and packs the 118-float normalisation
block that ``cp_sur_set`` takes.

The network covers the cells whose droplets cannot freeze (no droplets, or gas at
or above 273.15 K): growth and evaporation of droplets, deposition and
sublimation of crystals, nucleation away from its onset.  Freezing changes the
crystal number by orders of magnitude per kelvin and stays with the exact source
(the library's gate sends those cells there), so the training set holds only the
other regime.  In the step the library trusts a prediction whose every feature
increment stays within df_max (df_max_ice for the crystal moments) and whose
particle populations stay realizable; other cells take the exact source.

Features of a cell (computed on the device by ``cp_sur_features``, the same code
the in-step gate runs): f_v = asinh(U_v / s_in[v]) for the 15 conserved
variables, ln dt, log10 max(N_soot, 1).  Targets: for the particle moments
(v = 5..12) and the activated-soot number (v = 14), the increment of f_v over one
exact source integration, asinh(U'_v / s_in[v]) - f_v with U' = U + dt Q(U, dt);
the other outputs are trained to zero because the library closes them exactly
(water, gas mass, momentum and energy follow the condensate sources; soot
number is conserved).

The scales s_in put the asinh knee at a physical floor of each variable (one
particle per m^3 for the number moments, a 1 nm radius for the higher moments),
so a moment is log-scaled over its whole range.
"""
import math

import numpy as np

NET_VARS = (5, 6, 7, 8, 9, 10, 11, 12, 14)
S_IN = np.array([1.0, 100.0, 1.0, 1.0e5, 1.0e-3,
                 1.0, 1.0e-9, 1.0e-18, 1.0e-27,
                 1.0, 1.0e-9, 1.0e-18, 1.0e-27,
                 1.0, 1.0], dtype=np.float32)
N_IN, N_OUT = 17, 15
N_NORM = 15 + 4 * 17 + 2 * 15 + 5


class Dataset:
    """Rows of (features, target increments, ln S_l, dt) on the GPU."""

    def __init__(self, X, D, lnS, dt):
        self.X, self.D, self.lnS, self.dt = X, D, lnS, dt

    def __len__(self):
        return int(self.X.shape[0])

    def split(self, frac, seed=0):
        import torch
        g = torch.Generator(device="cpu").manual_seed(seed)
        p = torch.randperm(len(self), generator=g).to(self.X.device)
        k = int(round(frac * len(self)))
        a, b = p[k:], p[:k]
        pick = lambda idx: Dataset(self.X[idx].contiguous(), self.D[idx].contiguous(), self.lnS[idx].contiguous(),
                                   self.dt[idx].contiguous())
        return pick(a), pick(b)

    @staticmethod
    def cat(parts):
        import torch
        return Dataset(*[torch.cat([getattr(p, k) for p in parts]) for k in ("X", "D", "lnS", "dt")])


T_MELT = 273.15
N_MIN = 1.0


def collect(binding, cases, snapshots, every, dt_factors=(0.5, 1.0, 2.0), lnS_gate=0.05, warmup=0,
            precision=None, max_rows=None, seed=0, log=None, supersaturated=True):
    """Run each (mesh, case) on the GPU with the exact source and sample the cells
    whose source is non-zero, that lie away from liquid saturation
    (|ln S_l| >= lnS_gate) and whose droplets cannot freeze (the network's regime):
    ``snapshots`` samples, ``every`` steps apart, each at the CFL time step times
    every factor in dt_factors.  With max_rows, each sample keeps a seeded random
    subset so that the total stays near max_rows."""
    import torch
    precision = binding.CP_FP64 if precision is None else precision
    s_in = S_IN
    parts = []
    per_sample = None
    if max_rows:
        per_sample = max(1, int(max_rows) // (len(cases) * snapshots * len(dt_factors)))
    g = torch.Generator(device="cpu").manual_seed(seed)
    for ci, (m, c) in enumerate(cases):
        s = binding.Solver(m, c, precision)
        U = s.init()
        if warmup:
            s.step_n(U, warmup)
        for k in range(snapshots):
            s.step_n(U, every)
            dt0 = s.cfl_dt(U)
            Uf = U.reshape(15, -1).double()
            for fac in dt_factors:
                dt = dt0 * fac
                Q = s.source(U, dt).reshape(15, -1).double()
                F = s.sur_features(U, dt, s_in)
                no_freezing = (F[:, 18] >= T_MELT) | (Uf[5] <= N_MIN)
                act = (Q != 0).any(dim=0) & (F[:, 17].abs() >= lnS_gate) & no_freezing
                if not supersaturated:   # evaporation / sublimation / deposition only
                    act &= F[:, 17] <= -lnS_gate
                if not bool(act.any()):
                    continue
                if per_sample is not None:
                    idx = torch.nonzero(act).flatten()
                    if idx.numel() > per_sample:
                        keep = torch.randperm(idx.numel(), generator=g)[:per_sample].to(idx.device)
                        act = torch.zeros_like(act)
                        act[idx[keep]] = True
                Ua, Qa = Uf[:, act].t(), Q[:, act].t()
                sc = torch.tensor(s_in, dtype=torch.float64, device=U.device)
                D = torch.zeros_like(Ua)
                Up = torch.clamp(Ua + dt * Qa, min=0.0)
                for v in NET_VARS:
                    D[:, v] = torch.asinh(Up[:, v] / sc[v]) - torch.asinh(Ua[:, v] / sc[v])
                parts.append(Dataset(F[act, :17].contiguous(), D.float(), F[act, 17].contiguous(),
                                     torch.full((int(act.sum()),), dt, dtype=torch.float64, device=U.device)))
            if log:
                log("  case %d snapshot %d/%d: %d rows" % (ci, k + 1, snapshots,
                                                           int(parts[-1].X.shape[0]) if parts else 0))
        s.close()
    return Dataset.cat(parts)


class Norm:
    """Feature/target standardisation and the training envelope."""

    def __init__(self, data, lnS_gate=0.05, df_max=0.2, df_max_ice=0.01):
        import torch
        X, D = data.X.double(), data.D.double()
        self.s_in = S_IN.copy()
        self.mu_in = X.mean(0).cpu().numpy()
        sd = X.std(0).cpu().numpy()
        sd[sd < 1e-12] = 1.0
        self.sd_in = sd
        Z = (X - torch.tensor(self.mu_in, device=X.device)) / torch.tensor(self.sd_in, device=X.device)
        self.lo = Z.min(0).values.cpu().numpy()
        self.hi = Z.max(0).values.cpu().numpy()
        self.mu_out = np.zeros(N_OUT)
        self.sd_out = np.ones(N_OUT)
        for v in NET_VARS:
            self.mu_out[v] = float(D[:, v].mean())
            sdv = float(D[:, v].std())
            self.sd_out[v] = sdv if sdv > 1e-12 else 1.0
        self.lnS_gate = lnS_gate
        self.df_max = df_max
        self.df_max_ice = df_max_ice
        self.lnS_lo = float(data.lnS.min())
        self.lnS_hi = float(data.lnS.max())

    def pack(self):
        """The 118 floats of cp_sur_set, in the order the library reads them."""
        out = np.concatenate([self.s_in, self.mu_in, self.sd_in, self.lo, self.hi, self.mu_out, self.sd_out,
                              [self.lnS_gate, self.lnS_lo, self.lnS_hi, self.df_max,
                               self.df_max_ice]]).astype(np.float32)
        assert out.size == N_NORM
        return out

    def inputs(self, X):
        import torch
        mu = torch.tensor(self.mu_in, dtype=torch.float32, device=X.device)
        sd = torch.tensor(self.sd_in, dtype=torch.float32, device=X.device)
        return ((X - mu) / sd).contiguous()

    def targets(self, D):
        import torch
        mu = torch.tensor(self.mu_out, dtype=torch.float32, device=D.device)
        sd = torch.tensor(self.sd_out, dtype=torch.float32, device=D.device)
        return ((D - mu) / sd).contiguous()

    def decode(self, Y):
        import torch
        mu = torch.tensor(self.mu_out, dtype=torch.float32, device=Y.device)
        sd = torch.tensor(self.sd_out, dtype=torch.float32, device=Y.device)
        return Y * sd + mu


def init_params(seed, n_in=N_IN, n_h=256, n_out=N_OUT):
    """He initialisation (weights ~ N(0, 2/fan_in), zero biases), flat in the
    library's order W1, b1, W2, b2, W3, b3."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for a, b in ((n_in, n_h), (n_h, n_h), (n_h, n_out)):
        parts.append(g.normal(0.0, math.sqrt(2.0 / a), size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def train(binding, train_set, norm, epochs=30, batch=4096, lr=2e-3, lr_end=2e-5, warm_frac=0.03, seed=0,
          n_hidden=256, val_set=None, log=None):
    """Adam on the mean-squared error of the standardised targets, cosine learning
    rate with a linear warm-up; every pass of the network runs in the library's
    kernels.  Returns (network, history of (epoch, train loss, validation loss))."""
    import torch
    net = binding.MLP(N_IN, n_hidden, N_OUT)
    net.set_params(init_params(seed, N_IN, n_hidden, N_OUT))
    X = norm.inputs(train_set.X)
    T = norm.targets(train_set.D)
    n = X.shape[0]
    nb = max(1, n // batch)
    total = epochs * nb
    warm = max(1, int(warm_frac * total))
    g = torch.Generator(device="cpu").manual_seed(seed + 1)
    Xv = norm.inputs(val_set.X) if val_set is not None else None
    Tv = norm.targets(val_set.D) if val_set is not None else None
    hist = []
    it = 0
    for e in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        acc = 0.0
        for k in range(nb):
            idx = perm[k * batch:(k + 1) * batch]
            loss = net.loss_grad(X[idx].contiguous(), T[idx].contiguous())
            if it < warm:
                rate = lr * (it + 1) / warm
            else:
                q = (it - warm) / max(1, total - warm)
                rate = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * q))
            net.adam(rate)
            acc += loss
            it += 1
        vl = None
        if Xv is not None:
            vl = validation_loss(net, Xv, Tv)
        hist.append((e, acc / nb, vl))
        if log:
            log("  epoch %d: train %.4f%s" % (e, acc / nb, "" if vl is None else "  val %.4f" % vl))
    return net, hist


def validation_loss(net, Xs, Ts, chunk=65536):
    tot, n = 0.0, 0
    for a in range(0, Xs.shape[0], chunk):
        Y = net.forward(Xs[a:a + chunk].contiguous())
        tot += float(((Y - Ts[a:a + chunk]) ** 2).sum())
        n += Y.numel()
    return tot / max(n, 1)


def increment_errors(net, norm, data, chunk=65536):
    """Per output v in NET_VARS: median and 99th percentile of the relative error
    of the predicted new value U'_v (relative to max(|U'_v|, s_in[v]))."""
    import torch
    out = {}
    errs = {v: [] for v in NET_VARS}
    s = torch.tensor(norm.s_in, dtype=torch.float64, device=data.X.device)
    for a in range(0, len(data), chunk):
        X = data.X[a:a + chunk]
        Y = norm.decode(net.forward(norm.inputs(X))).double()
        f = X.double()
        D = data.D[a:a + chunk].double()
        for v in NET_VARS:
            # f_v carries FP32 rounding; the increment is exact in the targets
            Ut = s[v] * torch.sinh(torch.clamp(f[:, v] + D[:, v], min=0.0))
            Up = s[v] * torch.sinh(torch.clamp(f[:, v] + Y[:, v], min=0.0))
            errs[v].append(((Up - Ut).abs() / torch.clamp(Ut.abs(), min=float(s[v]))).cpu())
    for v in NET_VARS:
        e = torch.cat(errs[v]).numpy()
        out[v] = (float(np.median(e)), float(np.percentile(e, 99)))
    return out


def build(binding, cases, snapshots=40, every=20, epochs=30, lnS_gate=0.05, seed=0, val_frac=0.05, max_rows=None,
          batch=4096, lr=2e-3, df_max=0.2, df_max_ice=0.01, log=None, supersaturated=True):
    """Collect, fit the normalisation, train.  Returns (network, Norm, report).
    supersaturated=False trains on subsaturated cells only, so the envelope's ln S_l
    range keeps nucleating cells with the exact source too."""
    data = collect(binding, cases, snapshots, every, lnS_gate=lnS_gate, max_rows=max_rows, seed=seed, log=log,
                   supersaturated=supersaturated)
    tr, va = data.split(val_frac, seed)
    norm = Norm(tr, lnS_gate, df_max, df_max_ice)
    net, hist = train(binding, tr, norm, epochs=epochs, batch=batch, lr=lr, seed=seed, val_set=va, log=log)
    rep = {"rows": len(data), "train_rows": len(tr), "val_rows": len(va), "epochs": epochs,
           "first_val_loss": hist[0][2], "final_train_loss": hist[-1][1], "final_val_loss": hist[-1][2],
           "increment_errors": {str(v): e for v, e in increment_errors(net, norm, va).items()}}
    return net, norm, rep
