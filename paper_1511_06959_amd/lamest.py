"""Choice of the artificial-viscosity scale lambda from the growth of the adjoint energy.

The stabilised adjoint trades exactness for boundedness: without the added viscosity the adjoint
energy E_v^ of a chaotic flow grows exponentially in reverse time; with too much, the
sensitivities drift away from the true gradient ("Stabilizing adjoint equations"; "Results";
estimating the scaling factor for a given problem is left open in the "Conclusion").  This
module picks the smallest scale that stops the growth:

  1. run the primal window once and store it;
  2. run one homogeneous reverse sweep (no objective injection) per candidate
     lambda_k = f_k dx_min^2 from the same terminal adjoint, a seeded white-noise field that
     excites every mode, like the start of a power iteration; the candidates are members of one
     batched ensemble over the stored trajectory, so every reverse step is one launch per RK
     stage for all of them; E_v^ is recorded after every reverse step;
  3. fit the growth rate r_k of each sweep: the least-squares slope of log E_v^ against reverse
     time tau = (T - n) dt, over the part of the sweep after the first `skip` fraction (the decay
     of the grid-scale part of the noise);
  4. choose the smallest candidate with r_k <= target_rate (0: no growth) among those inside the
     explicit RK4 diffusion bound; optionally refine between it and the next smaller candidate
     by further sweeps at geometrically spaced scales.

The weights of the variable groups come from grid.nu_weight, so the estimate is the overall
scale for a fixed ratio between them.  Only scheduling and the fit (a few numbers per sweep) run
on the host; every step runs in the library's kernels.
"""
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import Ensemble, growth_sigma1

# explicit RK4 is stable on the negative real axis down to z = -2.785; the L_nu eigenvalues
# reach -nu sum_d 4 / dx_d^2
RK4_REAL_AXIS = 2.785


def growth_rate(E, dt, skip=0.25):
    """Least-squares slope of log E against reverse time.

    E: energies E[0..T] indexed by the step n of the state they belong to (E[T] is the terminal
    adjoint, E[0] the end of the reverse sweep); reverse time tau_n = (T - n) dt.  The first
    ceil(skip T) reverse steps are left out of the fit (the terminal transient)."""
    E = np.asarray(E, dtype=np.float64)
    T = len(E) - 1
    n0 = T - int(math.ceil(skip * T))  # fit over n = n0, ..., 0
    if n0 < 1:
        raise ValueError("the fit needs at least two energies after the skipped part")
    tau = (T - np.arange(n0 + 1)) * dt
    y = np.log(E[:n0 + 1])
    tm, ym = tau.mean(), y.mean()
    return float(((tau - tm) * (y - ym)).sum() / ((tau - tm) ** 2).sum())


def choose(factors, rates, stable, target_rate=0.0):
    """Index of the smallest stable candidate whose rate is <= target_rate (factors ascending),
    or None when there is none."""
    for k in range(len(factors)):
        if stable[k] and rates[k] <= target_rate:
            return k
    return None


def lambda_bound(g, sigma_max):
    """Largest lambda inside the explicit RK4 diffusion bound for the largest sigma_1."""
    wmax = max(g.nu_weight) if max(g.nu_weight) > 0.0 else 1.0
    s = sum(4.0 * (g.n[d] / g.L[d]) ** 2 for d in range(3))
    return RK4_REAL_AXIS / (wmax * max(sigma_max, 1e-300) * g.dt * s)


@dataclass
class Estimate:
    factor: float                  # chosen lambda / dx_min^2 (None: no candidate qualified)
    lam: float                     # chosen lambda (L^2)
    factors: list                  # every candidate tried, ascending
    rates: list                    # fitted growth rate of each (1/time)
    stable: list                   # inside the RK4 diffusion bound
    energies: dict = field(default_factory=dict)  # factor -> E[0..T]
    lam_max: float = None          # the RK4 diffusion bound of lambda on this window


class EnergySweeps:
    """The stored window of one box and batched homogeneous reverse sweeps over it."""

    def __init__(self, g, w0, s, nsteps, device):
        self.g, self.T, self.device = g, nsteps, device
        dt = g.dtype
        self.ens1 = Ensemble([g], [0], [0.0], None, device)
        ws = self.ens1.workspace(device)
        N5 = 5 * g.ncells
        self.s = None if s is None else torch.as_tensor(s).to(device=device, dtype=dt).reshape(-1)
        self.slots = [torch.empty(N5, dtype=dt, device=device) for _ in range(nsteps + 1)]
        self.slots[0].copy_(torch.as_tensor(w0).to(device=device, dtype=dt).reshape(-1))
        for t in range(nsteps):
            self.ens1.primal_step(1, self.slots[t], self.s, self.slots[t + 1], ws)

    def energies(self, lams, aT):
        """E[0..T] of one reverse sweep per lambda in lams, all from the terminal adjoint aT."""
        K, T = len(lams), self.T
        ens = Ensemble([self.g], [0] * K, list(lams), None, self.device)
        ws = ens.workspace(self.device)
        a = torch.zeros(5 * ens.offset(1, K), dtype=self.g.dtype, device=self.device)
        src = torch.as_tensor(aT).to(device=self.device, dtype=self.g.dtype).reshape(-1)
        for m in range(K):
            ens.member_slice(a, m).copy_(src)
        b = torch.zeros_like(a)
        E = torch.zeros((T + 1, K), dtype=torch.float64, device=self.device)
        ens.energy_vhat(K, self.slots[T], a, E[T], ws)
        for n in range(T - 1, -1, -1):
            ens.adjoint_step(K, self.slots[n], self.s, a, b, ws)
            a, b = b, a
            ens.energy_vhat(K, self.slots[n], a, E[n], ws)
        E = E.cpu().numpy()
        return [E[:, m].copy() for m in range(K)]


def estimate_lambda(g, w0, s, nsteps, factors=(0.0, 0.01, 0.03, 0.1, 0.3, 1.0), target_rate=0.0, skip=0.25,
                    refine=0, refine_points=4, aT=None, seed=0, device="cuda"):
    """Pick lambda for grid g and the window of nsteps RK4 steps from w0 (stored form, numpy or
    torch) with source s (or None).  factors: candidate lambda / dx_min^2.  aT: terminal adjoint
    (default: seeded standard normal).  refine: rounds of bisection between the chosen candidate
    and the next smaller one, each one batched sweep of refine_points scales spaced
    geometrically inside the bracket."""
    factors = sorted(float(f) for f in factors)
    dx2 = min(g.L[d] / g.n[d] for d in range(3)) ** 2
    if aT is None:
        aT = np.random.default_rng(seed).standard_normal(5 * g.ncells)
    sw = EnergySweeps(g, w0, s, nsteps, device)
    # sigma_1 at the first and last state of the window bounds the candidates
    sig = torch.empty(g.ncells, dtype=g.dtype, device=device)
    smax = 0.0
    for t in (0, nsteps):
        growth_sigma1(g, sw.slots[t], sig)
        smax = max(smax, float(sig.max()))
    lam_max = lambda_bound(g, smax)
    res = Estimate(None, None, [], [], [])

    def add(fs):
        for f, E in zip(fs, sw.energies([f * dx2 for f in fs], aT)):
            res.factors.append(f)
            res.rates.append(growth_rate(E, g.dt, skip))
            res.stable.append(f * dx2 <= lam_max)
            res.energies[f] = E
        order = np.argsort(res.factors)
        for name in ("factors", "rates", "stable"):
            setattr(res, name, [getattr(res, name)[i] for i in order])

    add(factors)
    k = choose(res.factors, res.rates, res.stable, target_rate)
    for _ in range(refine):
        if k is None or k == 0:
            break
        lo, hi = res.factors[k - 1], res.factors[k]
        lo = lo if lo > 0.0 else hi / 100.0
        add([float(x) for x in np.geomspace(lo, hi, refine_points + 2)[1:-1]])
        k = choose(res.factors, res.rates, res.stable, target_rate)
    if k is not None:
        res.factor = res.factors[k]
        res.lam = res.factor * dx2
    res.lam_max = lam_max
    return res
