"""Oracle states of the full-size workloads, sampled, for the GPU parity tests.

Calls only the CPU oracle (``oracle/``, built -O3 -march=native with OpenMP,
which computes the plain build's bits) and the seeded input generators
(``paper_1910_06059_amd.cases``).  Each file holds, per report step, p, s_w
and s_g at 4000 cells drawn with numpy's default_rng(0) (sorted), with the
Newton and linear iteration counts of the oracle run:

* ``c5_block_ilu0.npz``: the 100x100x50 waterflood of seed 5008, block ILU0
  on 4x4x50 columns (the GPU benchmark's preconditioner), three 10-day report
  steps, Newton CNV 1e-8 and MB 1e-11, BiCGStab to 1e-6;
* ``c4_largest.npz``: the three largest members of the 64-member ensemble
  (grids drawn with seed 4000), one 15-day report step each, ILU(0) of the
  whole member, the same tolerances.

Run from the repository root:  python tests/golden/make_golden.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1910_06059_amd import cases  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE = 4000


def sample(n):
    return np.sort(np.random.default_rng(0).choice(n, min(N_SAMPLE, n), replace=False))


def run(case, steps, blocks, so):
    m = oracle.Model(case, lib_path=so)
    if blocks:
        m.set_ilu_blocks(*blocks)
    idx = sample(m.n)
    y = case.initial_state()
    out = {"idx": idx.astype(np.int64), "p": [], "sw": [], "sg": [], "newton_its": [],
           "lin_its": []}
    for s, dt in enumerate(case.report_dt[:steps]):
        t0 = time.perf_counter()
        st, y, rep = m.advance(y, dt)
        if st != 0:
            raise RuntimeError(f"{case.name}: oracle step {s} failed ({st})")
        out["p"].append(y[idx, 0])
        out["sw"].append(y[idx, 1])
        out["sg"].append(y[idx, 2])
        out["newton_its"].append(rep.newton_its)
        out["lin_its"].append(rep.lin_its)
        print(f"{case.name} step {s}: {rep.newton_its} Newton, {rep.lin_its:.0f} linear, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    return {k: np.asarray(v) for k, v in out.items()}


def largest_members(k=3):
    sizes = [(cases.config4_member(m).n_active, m) for m in range(64)]
    return [m for _, m in sorted(sizes, reverse=True)[:k]]


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    so = oracle.build_baseline(os.path.join(HERE, "liboracle_golden.so"))
    oracle.set_threads(threads, so)
    c5 = cases.config5(5008)
    d = run(c5, 3, (4, 4, c5.nz), so)
    np.savez_compressed(os.path.join(HERE, "c5_block_ilu0.npz"), **d)
    members = largest_members()
    arrs = {"members": np.asarray(members)}
    for m in members:
        d = run(cases.config4_member(m), 1, None, so)
        for k, v in d.items():
            arrs[f"m{m}_{k}"] = v
    np.savez_compressed(os.path.join(HERE, "c4_largest.npz"), **arrs)
    os.remove(os.path.join(HERE, "liboracle_golden.so"))


if __name__ == "__main__":
    main()
