"""Learned droplet-shape surrogate on top of the batched lattice Boltzmann boxes.

The paper couples each droplet box to the velocity-gradient history A(t) seen
by a tracer (Sec. 3) and reads the droplet's shape from the semi-axes of its
inertia ellipsoid and the deformation D (Sec. 2 Eq. 4).  This module trains a
network that predicts those semi-axes from a window of recent A(t) samples,
with the full lattice Boltzmann box as its data source, its reference and
its fallback:

1. ``generate``: an ensemble of droplet boxes, each driven by its own A(t),
   runs in one launch per step (step loop replayed from a captured hipGraph,
   launch shape picked by the autotuner); every `stride` steps the droplet
   moments of all boxes are taken on the GPU.
2. ``make_windows``: window = the last 64 samples of A(t) (one every `stride`
   steps, oldest first); label = the three semi-axes over the droplet's
   volume-equivalent radius at the window's last sample (the shape; the size
   is set by the droplet volume, which the window does not carry).
3. ``train``: the network of ``mlp.Network`` (BF16 matrix-core kernels) with
   Adam on mini-batches drawn from device-resident data.
4. ``predict_with_fallback``: network inference in batches of 8192; windows
   whose predicted D exceeds the threshold are replayed through the batched
   lattice Boltzmann boxes instead (from a spherical droplet at the window's
   first sample, A(t) linear between samples), and those results replace the
   predictions.
5. ``mm_shapes``: the Maffettone-Minale model (Sec. 2 Eqs. 1, 2, 5) driven by
   the same A(t): the physical baseline the network must beat.

Every numerical step runs in the library's HIP kernels; this module moves
data, draws the (seeded) mini-batch order and times the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import Lattice, mm_integrate, sclbm_droplet_from_moments, sclbm_mm_semi_axes
from . import workloads as wl
from .mlp import NIN, Network, init_params

WINDOW = 64     # samples per window
STRIDE = 50     # lattice steps between samples
NCOMP = 9       # entries of A


@dataclass
class EnsembleRun:
    """Output of ``generate``: samples A_k (nbox, nsamp, 9) at times k * stride,
    droplet semi-axes (nbox, nsamp, 3, descending), volume-equivalent radii and
    deformation, plus the measured throughput."""
    n: int
    radius: float
    stride: int
    samples: np.ndarray
    semi_axes: np.ndarray
    r_eq: np.ndarray
    deformation: np.ndarray
    seconds: float
    lattice_updates: float
    launch: tuple = ()
    tables: list = field(default_factory=list, repr=False)

    @property
    def mlups(self) -> float:
        return self.lattice_updates / self.seconds / 1e6

    @property
    def lbm_samples_per_s(self) -> float:
        """One shape sample costs stride steps of one box."""
        return self.lattice_updates / self.seconds / (self.n ** 3 * self.stride)


def _stats_from_moments(mom, center, step):
    st = sclbm_droplet_from_moments(mom, center, step)
    return st["semi_axes"], st["r_eq"], st["deformation"]


def generate(case: wl.BoxCase, nsamp: int, *, autotune: bool = True, device="cuda:0", verbose=False) -> EnsembleRun:
    """Run the ensemble for (nsamp - 1) * stride steps and sample every stride steps."""
    import torch
    stride = case.stride
    steps = (nsamp - 1) * stride
    if stride % 2:
        raise ValueError("the captured step loop needs an even stride")
    nbox, n = case.nbox, case.n
    tabs = [np.asarray(t[:steps + 1]) for t in case.tables]
    if any(t.shape[0] < steps + 1 for t in tabs):
        raise ValueError("tables shorter than the run")
    lat = Lattice(n, n, n, nbox=nbox, bc="ghost", prec=case.prec, table_len=steps + 1, tau=(case.tau, case.tau),
                  g_ab=wl.G_AB, rho_b=case.rho_b, mach_max=wl.MACH_MAX * 1.05, device=device)
    for b in range(nbox):
        lat.set_gradient_table(tabs[b], 0, box=b)
    launch = lat.autotune(trial_steps=10) if autotune else lat.get_launch()
    for b in range(nbox):
        lat.init_droplet(lat.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
    mom = torch.empty((nsamp, nbox, 10), dtype=torch.float64, device=device)
    lat.droplet_moments_all(mom[0])
    lat.synchronize()
    t0 = time.perf_counter()
    for k in range(1, nsamp):
        lat.step_graph(stride)
        lat.droplet_moments_all(mom[k])
        if verbose and k % 50 == 0:
            lat.synchronize()
            print("  ensemble sample %d / %d (%.1f s)" % (k, nsamp - 1, time.perf_counter() - t0), flush=True)
    lat.synchronize()
    seconds = time.perf_counter() - t0
    m = mom.cpu().numpy()
    lat.close()
    axes = np.empty((nbox, nsamp, 3))
    req = np.empty((nbox, nsamp))
    dd = np.empty((nbox, nsamp))
    for b in range(nbox):
        for k in range(nsamp):
            axes[b, k], req[b, k], dd[b, k] = _stats_from_moments(m[k, b], lat.xc, k * stride)
    samples = np.stack([t[::stride][:nsamp] for t in tabs])
    return EnsembleRun(n=n, radius=case.radius, stride=stride, samples=samples, semi_axes=axes, r_eq=req,
                       deformation=dd, seconds=seconds, lattice_updates=float(n ** 3) * nbox * steps,
                       launch=tuple(launch[:3]), tables=tabs)


@dataclass
class WindowSet:
    windows: np.ndarray    # (m, 576) float32: 64 samples x 9, oldest first
    targets: np.ndarray    # (m, 3) float32: semi-axes / r_eq, descending
    box: np.ndarray        # (m,) source box
    k: np.ndarray          # (m,) sample index of the window's last sample


def make_windows(run: EnsembleRun, window: int = WINDOW) -> WindowSet:
    nbox, nsamp, _ = run.samples.shape
    ks = np.arange(window - 1, nsamp)
    w, t, bb, kk = [], [], [], []
    for b in range(nbox):
        for k in ks:
            w.append(run.samples[b, k - window + 1:k + 1].reshape(-1))
            t.append(run.semi_axes[b, k] / run.r_eq[b, k])
            bb.append(b)
            kk.append(k)
    return WindowSet(np.asarray(w, np.float32), np.asarray(t, np.float32), np.asarray(bb), np.asarray(kk))


def split_by_box(ws: WindowSet, every: int = 8, offset: int = 3):
    """Hold out whole trajectories: boxes b with b % every == offset validate."""
    val = (ws.box % every) == offset
    pick = lambda m: WindowSet(ws.windows[m], ws.targets[m], ws.box[m], ws.k[m])
    return pick(~val), pick(val)


DIAG = np.array([0, 4, 8])
OFFDIAG = np.array([1, 2, 3, 5, 6, 7])


def normalization(train: WindowSet, symmetric: bool = True):
    """Input shift/scale per entry of A (shared by the 64 lags) and mean/std of the
    targets.  With `symmetric` the statistics are those of the training set
    closed under the 48 cubic maps: the three diagonal entries share one
    mean and spread, the six off-diagonal ones share a spread about zero."""
    a = train.windows.reshape(-1, WINDOW, NCOMP).astype(np.float64)
    if symmetric:
        d = a[..., DIAG]
        md = d.mean()
        sd = np.sqrt(np.mean((d - md) ** 2))
        so = np.sqrt(np.mean(a[..., OFFDIAG] ** 2))
        mean = np.zeros(NCOMP)
        mean[DIAG] = md
        std = np.full(NCOMP, so)
        std[DIAG] = sd
    else:
        mean = a.mean(axis=(0, 1))
        std = a.std(axis=(0, 1))
    std[std == 0] = 1.0
    in_shift = np.tile(mean, WINDOW)
    in_scale = np.tile(1.0 / std, WINDOW)
    t = train.targets.astype(np.float64)
    out_shift = t.mean(axis=0)
    s = t.std(axis=0)
    s[s == 0] = 1.0
    return in_shift, in_scale, out_shift, 1.0 / s


@dataclass
class TrainResult:
    net: Network
    losses: list
    seconds: float
    steps: int


def train(train_set: WindowSet, *, steps: int = 10000, batch: int = 256, lr: float = 1e-3, lr_final: float = 1e-5,
          augment: bool = True, seed: int = 0, max_batch: int = 8192, device="cuda:0",
          net: Network = None) -> TrainResult:
    """Adam on the normalised MSE; the learning rate decays geometrically from lr
    to lr_final; mini-batch rows drawn without replacement per epoch and (with
    `augment`) each row mapped by a random one of the 48 cubic symmetries of the
    box, applied by the input kernel (all draws seeded, on the host)."""
    import torch
    if net is None:
        net = Network(max_batch=max(max_batch, batch), device=device)
        net.set_params(init_params(seed))
    net.set_normalization(*normalization(train_set, symmetric=augment))
    X = torch.from_numpy(train_set.windows).to(device)
    T = torch.from_numpy(train_set.targets).to(device)
    m = X.shape[0]
    rng = np.random.default_rng(seed + 1)
    order = np.concatenate([rng.permutation(m) for _ in range((steps * batch) // m + 2)]).astype(np.int32)
    idx_all = torch.from_numpy(order).to(device)
    sym_all = torch.from_numpy(rng.integers(0, 48, order.size).astype(np.int32)).to(device) if augment else None
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    losses = []
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for s in range(steps):
        idx = idx_all[s * batch:(s + 1) * batch]
        sym = sym_all[s * batch:(s + 1) * batch] if augment else None
        loss = net.train_step(X, T, idx, sym, lr=lr * decay ** s)
        if s % 100 == 0 or s == steps - 1:
            losses.append((s, float(loss.item())))
    torch.cuda.synchronize(device)
    return TrainResult(net, losses, time.perf_counter() - t0, steps)


def deformation(axes: np.ndarray) -> np.ndarray:
    a = np.sort(np.asarray(axes, dtype=np.float64), axis=-1)
    return (a[..., 2] - a[..., 0]) / (a[..., 2] + a[..., 0])


def replay(windows: np.ndarray, *, n: int, radius: float, stride: int = STRIDE, prec: str = "f32", max_boxes: int = 64,
           device="cuda:0"):
    """Lattice Boltzmann answer for each window: a spherical droplet at the first
    sample, A(t) linear between samples for (64 - 1) * stride steps, then the
    semi-axes over r_eq.  Returns (axes (m, 3), lattice updates)."""
    import torch
    windows = np.asarray(windows, dtype=np.float64).reshape(len(windows), -1, NCOMP)
    nwin = windows.shape[1]
    steps = (nwin - 1) * stride
    out = np.empty((len(windows), 3))
    lups = 0.0
    rho_b = wl.ghost_densities(radius)
    for s in range(0, len(windows), max_boxes):
        chunk = windows[s:s + max_boxes]
        nb = len(chunk)
        lat = Lattice(n, n, n, nbox=nb, bc="ghost", prec=prec, table_len=steps + 1, g_ab=wl.G_AB, rho_b=rho_b,
                      mach_max=0.0, device=device)
        for b in range(nb):
            tab = wl.per_step_table(chunk[b].reshape(-1, 3, 3), stride, steps + 1)
            lat.set_gradient_table(tab, 0, box=b)
            lat.init_droplet(lat.xc, radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0], box=b)
        lat.step_graph(steps) if steps % 2 == 0 else lat.step(steps)
        mom = torch.empty((nb, 10), dtype=torch.float64, device=device)
        lat.droplet_moments_all(mom)
        lat.synchronize()
        m = mom.cpu().numpy()
        for b in range(nb):
            ax, req, _ = _stats_from_moments(m[b], lat.xc, steps)
            out[s + b] = ax / req
        lups += float(n) ** 3 * nb * steps
        lat.close()
    return out, lups


@dataclass
class Prediction:
    axes: np.ndarray        # (m, 3)
    fallback: np.ndarray    # (m,) bool: replayed through the lattice Boltzmann boxes
    infer_seconds: float
    fallback_seconds: float
    fallback_lups: float


def predict_with_fallback(net: Network, windows: np.ndarray, *, threshold: float = 0.5, n: int = 64,
                          radius: float = 10.0, device="cuda:0") -> Prediction:
    import torch
    X = torch.from_numpy(np.ascontiguousarray(windows, dtype=np.float32)).to(device)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    Y = net.predict(X)
    torch.cuda.synchronize(device)
    t_inf = time.perf_counter() - t0
    axes = Y.cpu().numpy().astype(np.float64)
    fb = deformation(axes) > threshold
    t_fb, lups = 0.0, 0.0
    if fb.any():
        t1 = time.perf_counter()
        axes[fb], lups = replay(windows[fb], n=n, radius=radius, device=device)
        t_fb = time.perf_counter() - t1
    return Prediction(axes, fb, t_inf, t_fb, lups)


def mm_shapes(run: EnsembleRun, tau: float = wl.TAU, chi: float = 1.0, device="cuda:0") -> np.ndarray:
    """Maffettone-Minale semi-axes over R (det M = 1: the volume-equivalent radius
    is R) at every sample time, integrated from a sphere with the same A(t)
    tables as the boxes.  Shape (nbox, nsamp, 3), descending."""
    tau_d = wl.eta_s(tau) * run.radius / wl.SIGMA
    A = np.stack(run.tables)                                   # (nbox, steps + 1, 9)
    M = mm_integrate(A, tau_d, chi=chi, substeps=1, record_every=run.stride, device=device).cpu().numpy()
    return sclbm_mm_semi_axes(M)


def errors(pred: np.ndarray, truth: np.ndarray) -> dict:
    """Relative semi-axis errors |a_pred - a| / a over all windows and axes."""
    e = np.abs(np.asarray(pred, dtype=np.float64) - truth) / truth
    return dict(mean=float(e.mean()), rms=float(np.sqrt(np.mean(e * e))), p95=float(np.quantile(e, 0.95)),
                max=float(e.max()))


def inference_seconds(net: Network, batch: int = 8192, reps: int = 20, device="cuda:0", windows=None) -> float:
    """Average time of one inference batch: back-to-back sclmlp_predict calls
    through the C ABI on the network's stream, timed with HIP events on that
    stream (the Network.predict wrapper adds PyTorch stream synchronisation on
    the host around each call)."""
    import torch
    from .mlp import sclmlp_predict
    if windows is None:
        windows = np.random.default_rng(0).standard_normal((batch, NIN)).astype(np.float32) * 1e-3
    X = torch.from_numpy(np.ascontiguousarray(windows[:batch], dtype=np.float32)).to(device)
    out = torch.empty((X.shape[0], 3), dtype=torch.float32, device=device)
    net.predict(X, out)
    torch.cuda.synchronize(device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(reps):
        sclmlp_predict(net.ctx, X, X.shape[0], out)
    e1.record(net.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps
