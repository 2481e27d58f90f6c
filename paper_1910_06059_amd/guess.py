"""Training data, training loop and evaluation of the learned Newton guess.

Host-side sequencing of library calls only: the simulator steps
(opm_advance), the network's training steps (opm_guess_train_step) and the
guess-started report steps (opm_advance_guess) all run in the HIP kernels.
The network is trained on states the simulator itself produces: each sample
is one report step (y_{n-1}, y_n) -> y_{n+1}, n >= 1, of a seeded
realisation.
"""
from __future__ import annotations

import time
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import opm


def simulate(model: "opm.GpuModel", n_steps: Optional[int] = None, opts=None,
             log: Optional[Callable[[str], None]] = None):
    """States y_0 .. y_K over the case's report schedule (device tensors,
    starting from the initial state) and the per-step reports."""
    y = model.initial_state()
    states = [y.clone()]
    reps = []
    for k, dt in enumerate(model.case.report_dt[:n_steps]):
        t0 = time.perf_counter()
        st, rep = model.advance(y, dt, opts)
        if st != opm.OK:
            raise opm.OpmError(st, f"opm_advance step {k} of {model.case.name}")
        states.append(y.clone())
        d = rep.as_dict()
        d["wall"] = time.perf_counter() - t0
        reps.append(d)
        if log:
            log(f"{model.case.name} step {k}: newton {rep.newton_its} lin {rep.lin_its} "
                f"cuts {rep.cuts} {d['wall']:.2f}s")
    return states, reps


def sample_indices(n_states: int) -> List[Tuple[int, int, int]]:
    """(n, n-1, n+1) of every report step of a trajectory of n_states states
    that has a previous step (n >= 1): the network corrects the linear
    extrapolation of the last step, which the first step does not have."""
    return [(k, k - 1, k + 1) for k in range(1, n_states - 1)]


def train(net: "opm.GuessNet", data: Sequence[Tuple["opm.GpuModel", List[torch.Tensor]]],
          epochs: int, lr: float, lr_final: Optional[float] = None, seed: int = 0,
          log: Optional[Callable[[str], None]] = None) -> List[float]:
    """Adam over every sample of every trajectory, one sample per step,
    shuffled per epoch with a seeded generator; the step size decays
    geometrically from lr to lr_final.  Returns the mean loss per epoch."""
    rng = np.random.default_rng(seed)
    items = [(mi, tri) for mi, (_, states) in enumerate(data)
             for tri in sample_indices(len(states))]
    total = max(epochs * len(items) - 1, 1)
    dev = data[0][0].dev
    step = 0
    hist = []
    for e in range(epochs):
        losses = torch.zeros(len(items), dtype=torch.float64, device=dev)
        for j, idx in enumerate(rng.permutation(len(items))):
            mi, (a, b, c) = items[idx]
            model, states = data[mi]
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (step / total)
            model.guess_train_step(net, states[a], states[b], states[c], rate,
                                   loss_out=losses[j:j + 1])
            step += 1
        hist.append(float(losses.mean().cpu()))
        if log:
            log(f"epoch {e}: mean loss {hist[-1]:.4e}")
    return hist


def compare(model: "opm.GpuModel", net: Optional["opm.GuessNet"], n_steps: Optional[int] = None,
            opts=None, log: Optional[Callable[[str], None]] = None, keep: int = 0) -> dict:
    """Advance the case from its initial state, each report step after the
    first started from the learned guess (net given) or every step from the
    previous state (net None); the first step has no previous change and
    always starts from the previous state.
    Returns per-step Newton and linear iterations, wall time and the start
    taken (0 previous state, 1 learned guess, 2 its extrapolation path
    alone), the final state (host) and the states after the first `keep`
    report steps (host copies, taken outside the timed region)."""
    y = model.initial_state()
    y_nm1 = y.clone()
    out = {"newton": [], "lin": [], "wall": [], "used": [], "cuts": [], "states": []}
    for k, dt in enumerate(model.case.report_dt[:n_steps]):
        prev = y.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        use = net if k > 0 else None
        st, rep, used = model.advance_guess(y, y_nm1 if use is not None else None, dt, use, opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if st != opm.OK:
            raise opm.OpmError(st, f"opm_advance_guess step {k} of {model.case.name}")
        y_nm1 = prev
        out["newton"].append(rep.newton_its)
        out["lin"].append(rep.lin_its)
        out["wall"].append(wall)
        out["used"].append(used)
        out["cuts"].append(rep.cuts)
        if k < keep:
            out["states"].append(y.cpu().numpy())
        if log:
            log(f"{model.case.name} {'guess' if net is not None else 'prev '} step {k}: "
                f"newton {rep.newton_its} lin {rep.lin_its} used {used} {wall:.3f}s")
    out["final"] = y.cpu().numpy()
    return out
