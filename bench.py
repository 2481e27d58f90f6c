#!/usr/bin/env python3
"""Benchmark of the Newton linearisation and solve on one MI355X.

Workload: the 24x25x15 waterflood (9000 active cells, lognormal layered
permeability, one rate injector over the (0,0) column, four BHP producers),
FP64 state, ILU0-preconditioned BiCGStab to 1e-6, Newton to CNV 1e-8 / MB
1e-11.  One benchmark step is one 10-day implicit time step: every Newton
iteration assembles the residual and Jacobian by AD, tests convergence,
factors the preconditioner, solves with BiCGStab and applies the chopped
update, all in the HIP kernels of libopm_gpu.so.  Inputs are resident in HBM
before timing starts.  The preconditioner of `value` is the block ILU0 of
the paper's parallel runs (sec. 2.5, one block per subdomain; default 42
column subdomains of 4x4x15 cells, --ilu-blocks); the ILU(0) of the whole
system is timed on the same workload and reported beside it.

Metric: cell-Newton-iterations per second = sum over timed Newton iterations
of the active cell count / wall time of the timed steps.

Also printed on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes per launch / its
                average launch time (HIP events around repeated launches of
                the same kernel on the same stream, inside this run), against
                the 8 TB/s HBM peak;
  cpu_baseline  the CPU oracle (its plain FP64 C built -O3 -march=native with
                OpenMP assembly; the same bits as the test build) on a bounded
                sample of the same workload, on this machine's host cores,
                with all threads (value) and one (value_1thread).
"""
import argparse
import ctypes
import json
import subprocess
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-Newton-iterations/s (assembly+ILU0-BiCGStab) & % HBM roofline vs plain FP64"


def sweep_bytes_per_cell(precision: int) -> float:
    """Algorithmic bytes of one preconditioner application (forward plus
    backward sweep) per cell: three lower and three upper off-diagonal blocks
    read once, D^{-1} read in both sweeps, the right-hand side read, the
    result written by the forward sweep and updated by the backward sweep,
    plus the level-order index tables (perm twice, lower and upper positions)."""
    w = 8 if precision == 0 else 4
    blocks = (27 + 27) * w + 2 * 9 * w
    vectors = 24 + 24 + 24 + 24
    index = 4 * 2 + 12 + 12
    return blocks + vectors + index


def block_sweep_bytes_per_cell(precision: int) -> float:
    """Algorithmic bytes of one block-ILU0 preconditioner application per
    cell: the three lower and three upper off-diagonal blocks and D^{-1}
    (read in both sweeps) of the sweep records, the two 16-byte neighbour
    index records, the right-hand side read and the result written (the
    intermediate vector stays in LDS)."""
    w = 8 if precision == 0 else 4
    return (27 + 27 + 2 * 9) * w + 2 * 16 + 24 + 24


def spmv_bytes_per_cell(nnzb: int, n: int) -> float:
    """Algorithmic bytes of y = J x per block row: every 3x3 FP64 block and
    its column index once, the row pointer, x once and y once."""
    return (72 + 4) * nnzb / n + 4 + 24 + 24


def assemble_bytes(n: int, nnzb: int, nf: int) -> float:
    """Algorithmic bytes of one assembly: per cell the state, A0, pore volume,
    depth, row pointer and well pointer read and the residual written; per
    block the 3x3 FP64 block written and its column and face index read; per
    face the transmissibility read once."""
    return n * (24 + 24 + 8 + 8 + 4 + 4 + 24) + nnzb * (72 + 4 + 4) + nf * 8


def factor_bytes_per_cell(precision: int) -> float:
    """Algorithmic bytes of the ILU(0) factorisation per cell: the block row
    of J read once (7 FP64 blocks and their column indices), the level-order
    copies of the off-diagonal blocks and the inverse pivot written (27 + 27
    + 9 values, plus the FP64 pivot copy in mixed precision), and the three
    lower and three transposed blocks plus the neighbours' inverse pivots
    read again by the pivot recursion."""
    w = 8 if precision == 0 else 4
    pack = 7 * (72 + 4) + (27 + 27 + 9) * w + (72 if precision else 0)
    recurse = (27 + 27) * w + 3 * 9 * 8 + 9 * 8
    return pack + recurse


def block_factor_bytes_per_cell(precision: int) -> float:
    """Algorithmic bytes of the block-ILU0 factorisation per cell: the pivot
    recursion reads the diagonal, the three lower and the three transposed
    blocks of the row and writes D^{-1} (plus its FP32 copy); the record
    pass reads the six off-diagonal blocks and D^{-1} and writes the two
    sweep records and index records."""
    w = 8 if precision == 0 else 4
    recurse = 7 * 72 + 72 + (36 if precision else 0)
    records = 6 * 72 + 9 * w + 2 * 36 * w + 2 * 16
    return recurse + records


def gmres_cycle_bytes(n: int, nnzb: int, m: int, apply_bytes: float) -> float:
    """Bytes of one GMRes(m) call of one cycle as designed (x0 = 0, m
    iterations): x = 0 and ||b|| (b read, x written); the cycle-start
    residual SpMV (plus b read), its norm (v_0 read) and scaling (v_0 read
    and written); per iteration j the preconditioner solve (apply_bytes), the
    SpMV, then classical Gram-Schmidt applied twice, which reads the basis
    v_0 .. v_j three times (projections with w read; first update with w
    read and written; second update and norm with w read and written), and
    the next basis vector (w read, v_{j+1} written); the cycle ends with
    x += Z y (z_0 .. z_{m-1} read, x read and written)."""
    N8 = 24.0 * n
    spmv = spmv_bytes_per_cell(nnzb, n) * n
    total = 2 * N8 + (spmv + N8) + N8 + 2 * N8 + (m + 2) * N8
    for j in range(m):
        total += apply_bytes + spmv + 3 * (j + 1) * N8 + 7 * N8
    return total


def cpr_apply_bytes(levels, n: int, nnzb: int, apply_bytes: float) -> float:
    """Bytes of one CPR application as designed (one kernel per level down
    and up): down at level 0 the CSR values, columns and row pointers, the
    diagonal, the weights and r read, b_0 and the residual written; down at
    level l the CSR, the diagonal, the child lists and the finer residual
    read, b_l and the residual written; the coarsest level's child lists,
    finer residual and inverse read, its solution written; up at level l the
    CSR, the diagonal, b_l, the aggregate map and the coarser solution read,
    the level's solution written; the second-stage residual (the compact
    pressure column of J with its columns and row pointers, x_p and r read,
    r2 written); the ILU(0) solve (apply_bytes); z_p += x_p."""
    L = len(levels)
    total = 0.0
    for l in range(L - 1):
        nl, nnz = levels[l]
        csr = 12.0 * nnz + 4.0 * (nl + 1) + 8.0 * nl
        src = 48.0 * nl if l == 0 else 4.0 * (nl + 1) + 12.0 * levels[l - 1][0]
        total += csr + src + 16.0 * nl                                  # down
        total += csr + 8.0 * nl + 4.0 * nl + 8.0 * levels[l + 1][0] + 8.0 * nl   # up
    nc = levels[-1][0]
    src = 48.0 * nc if L == 1 else 4.0 * (nc + 1) + 12.0 * levels[-2][0]
    total += src + 8.0 * nc * nc + 8.0 * nc
    total += 28.0 * nnzb + 4.0 * (n + 1) + 8.0 * n + 48.0 * n   # second-stage residual
    return total + apply_bytes + 24.0 * n


def cpr_setup_bytes(levels, n: int, nnzb: int) -> float:
    """Bytes of one CPR setup as designed: the diagonal blocks and the
    pressure column of every block of J read with the pattern, weights,
    level-0 values and diagonal and the compact pressure column written;
    per coarse level its gather lists and the finer values read, its values
    and diagonal written; the coarsest matrix read and its inverse
    written."""
    total = (72.0 * n + 24.0 * nnzb + 4.0 * (n + 1) + 4.0 * n + 24.0 * n + 8.0 * nnzb + 8.0 * n +
             24.0 * nnzb)
    for l in range(1, len(levels)):
        nl, nnz = levels[l]
        total += 12.0 * levels[l - 1][1] + 4.0 * (nnz + 1) + 8.0 * nnz + 4.0 * nl + 8.0 * nl
    nc, nnzc = levels[-1]
    return total + 12.0 * nnzc + 8.0 * nc * nc


def parse_blocks(spec, case):
    """--ilu-blocks: 'none' (single block), 'BXxBY' (columns over the full
    depth) or 'BXxBYxBZ'."""
    if spec is None or spec == "none":
        return None
    parts = [int(v) for v in spec.lower().split("x")]
    if len(parts) == 2:
        parts.append(case.nz)
    return tuple(parts)


def measured_traffic(kernel_class: str, precision: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (profiles/counters.json, scaled by a plain
    256 MiB copy), or None when there is no record or one of the kernel's
    source files has changed since the counters were taken."""
    import hashlib
    tags = {("ilu0_apply", 0): "c2_fp64_ilu0_sweep", ("ilu0_apply", 1): "c2_mixed_ilu0_sweep",
            ("block_apply", 0): "c2_fp64_block_sweep", ("block_apply", 1): "c2_mixed_block_sweep"}
    tag = tags.get((kernel_class, precision))
    path = os.path.join(ROOT, "profiles", "counters.json")
    if tag is None or not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(tag)
    if not rec or not rec.get("traffic_bytes") or not rec.get("sources"):
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        p = os.path.join(ROOT, src)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return round(rec["traffic_bytes"]) if h.hexdigest()[:16] == rec.get("sources_sha256_16") else None


def _run_single(g, dt, steps, opts, opm):
    """Advance a single-system model over `steps` report steps; returns
    (wall seconds, cell-Newton-iterations, Newton its, linear its)."""
    import torch
    y = g.initial_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cni = newton = lin = 0
    for _ in range(steps):
        st, rep = g.advance(y, dt, opts)
        if st != opm.OK:
            raise RuntimeError(f"step failed: {opm._strerror(st)}")
        cni += rep.cell_newton_its
        newton += rep.newton_its
        lin += rep.lin_its
    torch.cuda.synchronize()
    return time.perf_counter() - t0, cni, newton, lin, y


def bench_mixed(args):
    """FP32 ILU(0) factors and sweeps inside FP64 BiCGStab against the plain
    FP64 GPU path on the masked 46x112x22 grid (about 45k active cells), same
    Newton (CNV 1e-8, MB 1e-11) and linear (1e-6) tolerances."""
    import numpy as np
    from paper_1910_06059_amd import cases, opm
    steps = args.steps or 10
    case = cases.config3()
    blk = parse_blocks(args.ilu_blocks, case)
    g = opm.GpuModel(case, ilu_blocks=blk)
    dt = case.report_dt[0]
    res = {}
    for prec in (0, 1):
        opts = opm.default_opts(case, precision=prec)
        _run_single(g, dt, 1, opts, opm)   # warm-up (kernel loading)
        wall, cni, newton, lin, y = _run_single(g, dt, steps, opts, opm)
        res[prec] = {"wall_s": round(wall, 4), "cell_newton_its_per_s": round(cni / wall, 1),
                     "newton_its": newton, "lin_its": lin, "state": y.cpu().numpy()}
    y64, y32 = res[0].pop("state"), res[1].pop("state")
    err_p = float(np.abs(y32[:, 0] - y64[:, 0]).max() / np.abs(y64[:, 0]).max())
    err_s = float(np.abs(y32[:, 1:] - y64[:, 1:]).max())
    vs_oracle = None
    if not args.no_cpu:
        # the oracle (its OpenMP build: the plain build's bits) over the same
        # report steps; both GPU runs' final states against it
        import oracle
        so = oracle.build_baseline()
        oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), so)
        m = oracle.Model(case, lib_path=so)
        yo = case.initial_state()
        for _ in range(steps):
            ost, yo, _ = m.advance(yo, dt)
            if ost != 0:
                raise RuntimeError("oracle step failed")
        vs_oracle = {}
        for name, yv in (("fp64", y64), ("mixed", y32)):
            vs_oracle[name] = {"p_rel": float(np.abs(yv[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()),
                               "s_abs": float(np.abs(yv[:, 1:] - yo[:, 1:]).max()),
                               "after_report_steps": steps}
    line = {"metric": "mixed-precision speedup over the plain FP64 GPU path (same tolerances)",
            "value": round(res[0]["wall_s"] / res[1]["wall_s"], 3), "unit": "x", "n_gpus": 1,
            "steps": steps, "warmup": 1, "higher_is_better": True, "dtype": "f64+f32-ilu",
            "data": "synthetic",
            "config": {"workload": f"46x112x22 masked grid, {g.n} active cells, 10-day steps",
                       "n_cells": g.n, "ilu_levels": g.n_levels,
                       "preconditioner": "ILU(0) of the whole system" if blk is None else
                       f"block ILU0, {g.pb.n_sub} column subdomains of {blk[0]}x{blk[1]}x{blk[2]}"},
            "fp64": res[0], "mixed": res[1],
            "mixed_vs_fp64_state": {"p_rel": err_p, "s_abs": err_s},
            "vs_fp64_oracle": vs_oracle}
    print(json.dumps(line), flush=True)


def c4_oracle_errors(ens, member_cases, dt):
    """Max pressure (relative) and saturation (absolute) differences of the
    three largest members after one report step from the oracle's states at
    4000 sampled cells each (tests/golden/c4_largest.npz, written by
    tests/golden/make_golden.py from the oracle alone).  Runs one untimed
    launch from the initial states."""
    import numpy as np
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "c4_largest.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    for t, m in zip(ens.y, ens.members):
        t.copy_(m.initial_state())
    ens.launch(dt, 1)
    torch.cuda.synchronize()
    states = ens.states()
    ep = es = 0.0
    for m in (int(v) for v in d["members"]):
        idx = d[f"m{m}_idx"]
        yo = np.stack([d[f"m{m}_p"][0], d[f"m{m}_sw"][0], d[f"m{m}_sg"][0]], axis=1)
        y = states[m][idx]
        ep = max(ep, float(np.abs(y[:, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()))
        es = max(es, float(np.abs(y[:, 1:] - yo[:, 1:]).max()))
    return {"p_rel": ep, "s_abs": es, "members": [int(v) for v in d["members"]],
            "report_steps": 1, "cells_per_member": int(len(d[f"m{int(d['members'][0])}_idx"]))}


def bench_ensemble(args):
    """64 members (uneven grids 20..60 x 20..60 x 20..30) advanced 20 report
    steps of 15 days in one persistent launch (replayed from a captured
    graph, launch shape picked by the autotuner beforehand: with the members
    built on a block-ILU0 topology of whole-column subdomains, as many
    workgroups as the device has compute units, shared out in proportion to
    the members' rows), against the single-system FP64 GPU path run member by
    member on a sample of members, and against one workgroup per member."""
    import torch
    from paper_1910_06059_amd import cases, opm
    steps = args.steps or 20
    nm = args.members
    member_cases = [cases.config4_member(m) for m in range(nm)]
    dt = member_cases[0].report_dt[0]
    split = None if args.member_split == "none" else tuple(int(v) for v in args.member_split.split("x"))
    # warm-up: load the kernels on a two-member ensemble
    warm = opm.Ensemble([cases.box_case(4, 4, 3, seed=1), cases.box_case(3, 5, 2, seed=2)],
                        precision=opm.PREC_MIXED)
    warm.launch(dt, 1)
    torch.cuda.synchronize()
    out = {}
    for prec in (opm.PREC_MIXED, opm.PREC_FP64):
        ens = opm.Ensemble(member_cases, precision=prec, member_split=split)
        # launch shape from the autotuner (untimed: one trial report step per
        # shape, states restored afterwards), then the timed work as one
        # captured graph holding the single persistent launch
        tuning = ens.autotune(dt, cache=args.tuning_cache)
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            with torch.cuda.graph(graph, stream=cap):
                ens.launch(dt, steps)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        reps = ens.read_reports()
        ok = sum(1 for r in reps if r["status"] == 0 and r["steps_done"] == steps)
        out[prec] = {"wall_s": round(wall, 3), "members_steps_per_s": round(nm * steps / wall, 3),
                     "members_ok": ok,
                     "newton_its": sum(r["newton_its"] for r in reps),
                     "lin_its": sum(r["lin_its"] for r in reps),
                     "cell_newton_its_per_s": round(sum(r["cell_newton_its"] for r in reps) / wall, 1),
                     "launch_shape": tuning}
        if nm == 64:
            out[prec]["vs_fp64_oracle"] = c4_oracle_errors(ens, member_cases, dt)
        del ens, graph
    # one workgroup per member (each member's ILU(0) of the whole system), FP32
    # factors, the same report steps: what the split launch is measured against
    ref_steps = min(steps, args.one_wg_steps)
    one = None
    if split is not None and ref_steps > 0:
        ens = opm.Ensemble(member_cases, precision=opm.PREC_MIXED)
        tuning = ens.autotune(dt, cache=args.tuning_cache)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.launch(dt, ref_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        reps = ens.read_reports()
        one = {"members_steps_per_s": round(nm * ref_steps / wall, 3), "steps": ref_steps,
               "members_ok": sum(1 for r in reps if r["status"] == 0 and r["steps_done"] == ref_steps),
               "launch_shape": tuning}
        del ens
    # single-system FP64 path, member by member, on a sample spread over sizes
    order = sorted(range(nm), key=lambda m: member_cases[m].n_active)
    k = max(1, min(args.baseline_members, nm))
    sample = [order[int(round(i * (nm - 1) / max(1, k - 1)))] for i in range(k)]
    base_steps = min(steps, 2)
    bwall = 0.0
    for m in sample:
        g = opm.GpuModel(member_cases[m])
        opts = opm.default_opts(member_cases[m], precision=opm.PREC_FP64)
        _run_single(g, dt, 1, opts, opm)
        wall, *_ = _run_single(g, dt, base_steps, opts, opm)
        bwall += wall
    base_rate = len(sample) * base_steps / bwall
    line = {"metric": "ensemble members-steps/s (one persistent launch) and speedup over the "
                      "single-system FP64 GPU path", "value": out[opm.PREC_MIXED]["members_steps_per_s"],
            "unit": "members-steps/s", "n_gpus": 1, "steps": steps, "warmup": 1,
            "higher_is_better": True, "dtype": "f64+f32-ilu", "data": "synthetic",
            "config": {"workload": f"{nm} members, grids 20..60 x 20..60 x 20..30, 15-day steps",
                       "total_cells": sum(c.n_active for c in member_cases),
                       "member_preconditioner": ("ILU(0) of the whole member" if split is None else
                                                 f"block ILU0 on {split[0]}x{split[1]} whole-column "
                                                 "subdomains per member")},
            "ensemble_mixed": out[opm.PREC_MIXED], "ensemble_fp64": out[opm.PREC_FP64],
            "one_workgroup_per_member_mixed": one,
            "speedup_vs_one_workgroup_per_member": (round(out[opm.PREC_MIXED]["members_steps_per_s"] /
                                                          one["members_steps_per_s"], 2)
                                                    if one else None),
            "single_system_fp64": {"members_steps_per_s": round(base_rate, 4),
                                   "sample": f"members {sample}, first {base_steps} steps each"},
            "speedup_vs_single_fp64": round(out[opm.PREC_MIXED]["members_steps_per_s"] / base_rate, 2),
            "speedup_fp64_ensemble_vs_single_fp64": round(out[opm.PREC_FP64]["members_steps_per_s"] / base_rate, 2)}
    print(json.dumps(line), flush=True)


def oracle_sampled_errors(runs):
    """Max pressure (relative) and saturation (absolute) differences of the
    first report steps of the 500k-cell seed-5008 runs from the oracle's
    states at its 4000 sampled cells (tests/golden/c5_block_ilu0.npz, written
    by tests/golden/make_golden.py from the oracle alone)."""
    import numpy as np
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "c5_block_ilu0.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    idx = d["idx"]
    out = {}
    for name, states in runs.items():
        ep = es = 0.0
        for s, y in enumerate(states[:len(d["p"])]):
            yo = np.stack([d["p"][s], d["sw"][s], d["sg"][s]], axis=1)
            ep = max(ep, float(np.abs(y[idx, 0] - yo[:, 0]).max() / np.abs(yo[:, 0]).max()))
            es = max(es, float(np.abs(y[idx, 1:] - yo[:, 1:]).max()))
        out[name] = {"p_rel": ep, "s_abs": es, "report_steps": min(len(states), len(d["p"])),
                     "cells": int(len(idx))}
    return out


def bench_guess(args):
    """Learned Newton initial guess on the 100x100x50 waterflood (500k active
    cells, lognormal permeability median 100 mD and sigma_ln 2, four water
    injectors, five BHP producers, 10-day report steps).  The network trains
    on the report steps that the FP64 GPU simulator produces for the
    training seeds; each held-out seed is then advanced three ways at the same
    Newton (CNV 1e-8, MB 1e-11) and linear (1e-6) tolerances: from the
    previous state, from the linear extrapolation y_n + (y_n - y_{n-1}) alone
    (the network's skip path with a zero correction), and from the learned
    guess (each step taking the lowest-CNV start among the previous state,
    the learned guess and its extrapolation path alone).  The first report
    step of every run starts from the previous state (it has no previous
    change)."""
    import numpy as np
    import torch
    from paper_1910_06059_amd import cases, guess, opm
    steps = args.steps or 25
    train_seeds = list(range(5000, 5000 + args.train_seeds))
    test_seeds = [5008, 5009][:args.test_seeds]

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    data = []
    gen_newton = 0
    blk = parse_blocks(args.ilu_blocks, cases.config5(train_seeds[0]))
    for seed in train_seeds:
        g = opm.GpuModel(cases.config5(seed), ilu_blocks=blk)
        states, reps = guess.simulate(g, steps, log=log)
        gen_newton += sum(r["newton_its"] for r in reps)
        g._work.clear()            # training needs the problem and the states only
        data.append((g, states))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    net = opm.GuessNet(seed=0)
    t0 = time.perf_counter()
    hist = guess.train(net, data, epochs=args.epochs, lr=args.lr, lr_final=0.1 * args.lr,
                       log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples = sum(len(guess.sample_indices(len(st))) for _, st in data)
    if args.save_net:
        np.save(args.save_net, net.params())
    del data
    torch.cuda.empty_cache()
    zero = opm.GuessNet(np.zeros(opm.GUESS_PARAMS, np.float32))
    runs = {"previous_state": None, "extrapolation": zero, "learned": net}
    tot = {k: {"wall_s": 0.0, "newton_its": 0, "lin_its": 0, "guess_starts": 0,
               "learned_starts": 0, "extrapolation_starts": 0} for k in runs}
    per_seed = {}
    state_diff = 0.0
    vs_oracle = None
    for seed in test_seeds:
        g = opm.GpuModel(cases.config5(seed), ilu_blocks=blk)
        out = {}
        for name, n_ in runs.items():
            r = guess.compare(g, n_, steps, log=log, keep=3 if seed == 5008 else 0)
            out[name] = r
            t = tot[name]
            t["wall_s"] += sum(r["wall"])
            t["newton_its"] += sum(r["newton"])
            t["lin_its"] += sum(r["lin"])
            t["guess_starts"] += sum(1 for u in r["used"] if u)
            t["learned_starts"] += sum(1 for u in r["used"] if u == 1)
            t["extrapolation_starts"] += sum(1 for u in r["used"] if u == 2)
        base = out["previous_state"]["final"]
        for name in ("extrapolation", "learned"):
            f = out[name]["final"]
            state_diff = max(state_diff, float(np.max(np.abs(f[:, 0] - base[:, 0]) / np.abs(base[:, 0]))),
                             float(np.max(np.abs(f[:, 1:] - base[:, 1:]))))
        per_seed[seed] = {k: {"newton": v["newton"], "used": v["used"]} for k, v in out.items()}
        if seed == 5008:
            vs_oracle = oracle_sampled_errors({k: v["states"] for k, v in out.items()})
    # inference cost: HIP events around repeated opm_guess_infer on the last test model
    y = g.initial_state()
    yg = g.zeros_state()
    stream = torch.cuda.current_stream()
    for _ in range(3):
        g.guess_infer(net, y, y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 50
    s_work = net.struct(g)
    L = opm._guess_lib()
    import ctypes
    work = g.workspace("guess", L.opm_guess_work_bytes(g._pbp(), ctypes.byref(s_work)))
    e0.record(stream)
    for _ in range(reps):
        L.opm_guess_infer(g._pbp(), ctypes.byref(s_work), opm._ptr(y), opm._ptr(y), opm._ptr(yg),
                          opm._ptr(work), opm._stream())
    e1.record(stream)
    e1.synchronize()
    t_inf = e0.elapsed_time(e1) * 1e-3 / reps
    nbox = g.case.n_box
    flops = 3 * 2 * 27 * 16 * 16 * nbox
    pt = tot["previous_state"]
    et, lt = tot["extrapolation"], tot["learned"]
    eligible = (steps - 1) * len(test_seeds)
    line = {"metric": "learned Newton guess: speedup over the previous-state start (wall time of "
                      "the held-out runs, same tolerances)",
            "value": round(pt["wall_s"] / tot["learned"]["wall_s"], 4), "unit": "x",
            "n_gpus": 1, "steps": steps, "warmup": 0, "higher_is_better": True,
            "dtype": "f64 (simulator) + bf16/f32 (network)", "data": "synthetic",
            "config": {"workload": f"100x100x50 waterflood, {g.n} cells, 10-day steps, "
                                   f"train seeds {train_seeds[0]}-{train_seeds[-1]}, "
                                   f"test seeds {test_seeds}",
                       "preconditioner": "ILU(0) of the whole system" if blk is None else
                       f"block ILU0, {g.pb.n_sub} column subdomains of {blk[0]}x{blk[1]}x{blk[2]}"},
            "runs": tot,
            "speedup_extrapolation": round(pt["wall_s"] / tot["extrapolation"]["wall_s"], 4),
            "newton_its_ratio_learned": round(tot["learned"]["newton_its"] / pt["newton_its"], 4),
            "newton_its_ratio_extrapolation": round(tot["extrapolation"]["newton_its"] / pt["newton_its"], 4),
            "max_state_difference_vs_previous_state_start": state_diff,
            "learned_vs_extrapolation": {
                "speedup": round(et["wall_s"] / lt["wall_s"], 4),
                "newton_its_ratio": round(lt["newton_its"] / et["newton_its"], 4),
                "lin_its_ratio": round(lt["lin_its"] / et["lin_its"], 4),
                "learned_chosen": lt["learned_starts"], "eligible_steps": eligible,
                "learned_chosen_fraction": round(lt["learned_starts"] / max(eligible, 1), 4)},
            "extrapolation_vs_previous_state": {
                "speedup": round(pt["wall_s"] / et["wall_s"], 4),
                "newton_its_ratio": round(et["newton_its"] / pt["newton_its"], 4)},
            "vs_fp64_oracle": vs_oracle,
            "training": {"samples": n_samples, "epochs": args.epochs, "lr": args.lr,
                         "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
                         "train_s": round(t_train, 2), "data_generation_s": round(t_gen, 2),
                         "data_generation_newton_its": gen_newton},
            "inference": {"us_per_call": round(t_inf * 1e6, 2),
                          "conv_tflops": round(flops / t_inf / 1e12, 2),
                          "frac_of_bf16_mfma_peak": round(flops / t_inf / 2.5e15, 5)},
            "per_seed": per_seed}
    print(json.dumps(line), flush=True)


def bench_kernels(args):
    """Per-kernel HBM roofline on the 100x100x50 system (500k cells, 3.46M
    blocks), where the data no longer fits the caches: HIP-event timing of
    repeated launches (on the launch stream) of the BSR SpMV, the ILU(0)
    application with FP64 and FP32 factors, the assembly and the ILU(0)
    factorisation, each divided into its algorithmic bytes."""
    import numpy as np
    import torch
    from paper_1910_06059_amd import cases, opm
    nx, ny, nz = (int(v) for v in args.kernel_grid.lower().split("x"))
    case = cases.config5(5008, nx, ny, nz)
    g = opm.GpuModel(case)
    dt = case.report_dt[0]
    y = g.initial_state()
    acc0 = g.accumulation(y)
    yk = y.clone()
    yk[:, 0] += 1e4
    R, J, _ = g.assemble(yk, acc0, dt)
    ilu = {p: g.ilu0_factor(J, p)[0] for p in (0, 1)}
    blk = parse_blocks(args.ilu_blocks, case) or (4, 4, case.nz)
    gb = opm.GpuModel(case, ilu_blocks=blk)
    Jb_ = J.clone()   # same cell numbering and pattern: the same Jacobian
    bilu = {p: gb.ilu0_factor(Jb_, p)[0] for p in (0, 1)}
    pbb = gb._pbp()
    x = g.zeros_state()
    L = opm.lib()
    pbp = g._pbp()
    sp = opm._ptr
    st = opm._stream()
    stream = torch.cuda.current_stream()
    reps = args.kernel_reps

    def timed(fn):
        for _ in range(3):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    if args.copy_probe_mb > 0:
        src = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device=g.dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = g.n
    norms = torch.zeros(L.opm_norms_bytes(pbp) // 8, dtype=torch.float64, device=g.dev)
    Rb, Jb = torch.empty_like(R), torch.empty_like(J)
    status = torch.zeros(1, dtype=torch.int32, device=g.dev)
    ilu_tmp = {p: torch.empty_like(ilu[p]) for p in (0, 1)}
    kern = {
        "spmv": (lambda: L.opm_spmv(pbp, sp(J), sp(R), sp(x), st),
                 spmv_bytes_per_cell(g.nnzb, n) * n, "k_spmv"),
        "ilu0_apply_fp64": (lambda: L.opm_ilu0_apply(pbp, sp(ilu[0]), 0, sp(R), sp(x), st),
                            sweep_bytes_per_cell(0) * n,
                            "k_plane_reset + k_sweep_planes forward and backward (FP64)"),
        "ilu0_apply_fp32": (lambda: L.opm_ilu0_apply(pbp, sp(ilu[1]), 1, sp(R), sp(x), st),
                            sweep_bytes_per_cell(1) * n,
                            "k_plane_reset + k_sweep_planes forward and backward (FP32)"),
        "assemble": (lambda: L.opm_assemble(pbp, sp(yk), sp(acc0), dt, sp(Rb), sp(Jb), sp(norms), st),
                     assemble_bytes(n, g.nnzb, g.nf), "k_assemble_tiled + k_norms_final"),
        "ilu0_factor_fp64": (lambda: L.opm_ilu0_factor(pbp, sp(J), sp(ilu_tmp[0]), 0, sp(status), st),
                             factor_bytes_per_cell(0) * n,
                             "k_pack + k_plane_init + k_plane_fill + k_plane_factor_reset + "
                             "k_factor_planes + k_pack_records (FP64)"),
        "block_apply_fp64": (lambda: L.opm_ilu0_apply(pbb, sp(bilu[0]), 0, sp(R), sp(x), st),
                             block_sweep_bytes_per_cell(0) * n,
                             f"k_apply_blocks (FP64, {gb.pb.n_sub} subdomains of {blk})"),
        "block_apply_fp32": (lambda: L.opm_ilu0_apply(pbb, sp(bilu[1]), 1, sp(R), sp(x), st),
                             block_sweep_bytes_per_cell(1) * n,
                             f"k_apply_blocks (FP32, {gb.pb.n_sub} subdomains of {blk})"),
        "block_factor_fp64": (lambda: L.opm_ilu0_factor(pbb, sp(Jb_), sp(ilu_tmp[0]), 0, sp(status), st),
                              block_factor_bytes_per_cell(0) * n,
                              "k_factor_blocks + k_pack_block_records (FP64)"),
    }
    # assembly with live oil on the same grid: a seeded state, half of the
    # cells with free gas (x = s_g), half undersaturated (x = r_go < r_s(p))
    case_l = cases.config5(5008, nx, ny, nz)
    case_l.fluid = cases.live_fluid()
    gl = opm.GpuModel(case_l)
    rng = np.random.default_rng(7)
    mean_l = rng.integers(0, 2, gl.n).astype(np.uint8)
    yl = np.empty((gl.n, 3))
    yl[:, 0] = 3000 * cases.PSI + rng.uniform(-200, 200, gl.n) * cases.PSI
    yl[:, 1] = rng.uniform(0.15, 0.4, gl.n)
    yl[:, 2] = np.where(mean_l == 0, rng.uniform(0.02, 0.2, gl.n),
                        rng.uniform(0.3, 0.9, gl.n) * case_l.fluid.rs_c * yl[:, 0])
    gl.set_meaning(mean_l)
    yl_t = gl.state(yl)
    acc_l = gl.accumulation(yl_t)
    Rl, Jl = torch.empty_like(R), torch.empty_like(J)
    norms_l = torch.zeros(L.opm_norms_bytes(gl._pbp()) // 8, dtype=torch.float64, device=g.dev)
    pbl = gl._pbp()
    kern["assemble_live"] = (
        lambda: L.opm_assemble(pbl, sp(yl_t), sp(acc_l), dt, sp(Rl), sp(Jl), sp(norms_l), st),
        assemble_bytes(n, g.nnzb, g.nf) + n, "k_assemble<live> + k_norms_final (live oil)")
    # one GMRes(m) cycle with the FP64 block ILU0 (rtol 0: exactly m iterations)
    m = args.restart
    gwork = torch.empty(L.opm_gmres_bytes(pbb, m), dtype=torch.uint8, device=g.dev)
    grep = opm.SolveReport()
    xg = g.zeros_state()
    kern["gmres_cycle"] = (
        lambda: L.opm_gmres(pbb, sp(Jb_), sp(bilu[0]), 0, sp(R), sp(xg), 0.0, m, m, sp(gwork),
                            ctypes.byref(grep), st),
        gmres_cycle_bytes(n, g.nnzb, m, block_sweep_bytes_per_cell(0) * n),
        f"one GMRes({m}) cycle: {m} x (k_apply_blocks + k_gm_spmv + k_gm_dots + k_gm_cgs1 + "
        "k_gm_cgs2 + k_gm_rotate) + start and finish kernels (FP64 block ILU0)")
    # CPR-AMG on the same system (FP64 block ILU0 as its second stage)
    cpr_k, cpr_st = gb.cpr_setup(Jb_)
    lv = gb.amg_levels()
    kern["cpr_setup"] = (
        lambda: L.opm_cpr_setup(pbb, sp(Jb_), sp(cpr_k), sp(cpr_st), st),
        cpr_setup_bytes(lv, n, g.nnzb),
        f"k_cpr_weights + {len(lv) - 1} x (k_cpr_galerkin + k_cpr_diag) + k_cpr_inverse")
    kern["cpr_apply"] = (
        lambda: L.opm_cpr_apply(pbb, sp(Jb_), sp(bilu[0]), 0, sp(cpr_k), sp(R), sp(x), st),
        cpr_apply_bytes(lv, n, g.nnzb, block_sweep_bytes_per_cell(0) * n),
        f"V(1,1) cycle over {len(lv)} levels ({'/'.join(str(a) for a, _ in lv)} unknowns: "
        f"{len(lv) - 1} x k_cpr_down + k_cpr_coarse + {len(lv) - 1} x k_cpr_up) + k_cpr_r2 + "
        "k_apply_blocks (FP64) + k_cpr_add")
    # a whole linear solve (BiCGStab to 1e-6) with either preconditioner: the
    # iterations CPR saves against its dearer application
    kwork = torch.empty(L.opm_krylov_bytes(pbb), dtype=torch.uint8, device=g.dev)
    srep = {"ilu0": opm.SolveReport(), "cpr": opm.SolveReport()}
    xs = g.zeros_state()
    kern["solve_block_ilu0"] = (
        lambda: L.opm_bicgstab(pbb, sp(Jb_), sp(bilu[0]), 0, sp(R), sp(xs), 1e-6, 1000,
                               sp(kwork), ctypes.byref(srep["ilu0"]), st),
        0, "BiCGStab to 1e-6 with the FP64 block ILU0 (whole solve)")
    kern["solve_cpr"] = (
        lambda: L.opm_bicgstab_cpr(pbb, sp(Jb_), sp(bilu[0]), 0, sp(cpr_k), sp(R), sp(xs), 1e-6,
                                   1000, sp(kwork), ctypes.byref(srep["cpr"]), st),
        0, "BiCGStab to 1e-6 with CPR-AMG + FP64 block ILU0 (whole solve)")
    if args.kernels:
        keep = set(args.kernels.split(","))
        kern = {k: v for k, v in kern.items() if k in keep}
    res = {}
    for name, (fn, nbytes, kname) in kern.items():
        t = timed(fn)
        res[name] = {"kernel": kname, "us": round(t * 1e6, 2), "bytes": int(nbytes),
                     "gbs": round(nbytes / t / 1e9, 1), "frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4)}
        if name.startswith("solve_"):
            rp_ = srep["ilu0" if name == "solve_block_ilu0" else "cpr"]
            res[name] = {"kernel": kname, "us": round(t * 1e6, 2), "its": rp_.its,
                         "half": rp_.half, "status": rp_.status}
            continue
        if name == "gmres_cycle":
            assert grep.its == m and grep.status == opm.ENOTCONV, (grep.its, grep.status)
            res[name]["us_per_iteration"] = round(t * 1e6 / m, 2)
    line = {"metric": f"kernel HBM roofline on the {n}-cell system (algorithmic bytes / HIP-event "
                      "time per launch)", "value": res.get("spmv", {}).get("frac"),
            "unit": "fraction of 8 TB/s (SpMV)", "n_gpus": 1, "steps": reps, "warmup": 3,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{nx}x{ny}x{nz} system, {n} cells, {g.nnzb} blocks, "
                                   f"{g.n_levels} ILU levels (max {g.max_level} rows), block ILU0 "
                                   f"on {gb.pb.n_sub} subdomains of {blk[0]}x{blk[1]}x{blk[2]}"},
            "kernels": res}
    print(json.dumps(line), flush=True)


def host_cpu():
    """nproc and the lscpu model name of the host running the CPU baseline."""
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "lscpu_model": model}


def cpu_baseline(case, dt, opts, seconds):
    """The oracle (plain FP64 C, its own sources) built for the host with
    -O3 -march=native and OpenMP (assembly over cells and faces and the
    Jacobian product over rows in parallel, the same bits as the plain
    build; ILU(0) and BiCGStab serial, the paper's serial default), timed on
    report steps of the same workload with one thread and with all the
    threads OpenMP is given; about `seconds` of CPU work each."""
    import oracle
    so = oracle.build_baseline()
    oopts = oracle.default_opts(case, krylov=int(opts.krylov), restart=int(opts.restart),
                                precond=int(opts.precond))
    all_threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                                     so)

    def timed(threads):
        oracle.set_threads(threads, so)
        m = oracle.Model(case, lib_path=so)

        def restart():
            m.set_meaning(case.initial_meaning())
            if case.standard_wells:
                m.set_well_state(case.standard_well_init()[1])
            return case.initial_state()

        yo = restart()
        c_cni, c_wall, c_steps = 0.0, 0.0, 0
        while c_wall < seconds:
            t1 = time.perf_counter()
            ost, yo, orep = m.advance(yo, dt, oopts)
            c_wall += time.perf_counter() - t1
            if ost != 0:
                break
            c_cni += orep.cell_newton_its
            c_steps += 1
            if c_steps % len(case.report_dt) == 0:   # schedule done: start it again
                yo = restart()
        return c_cni / c_wall, c_steps, c_wall

    v1, s1, w1 = timed(1)
    vn, sn, wn = timed(all_threads)
    days = round(dt / 86400)
    return {"value": round(vn, 1), "unit": "cell-Newton-iterations/s", "cores": all_threads,
            "kind": "oracle", "value_1thread": round(v1, 1), "host": host_cpu(),
            "sample": f"{sn} {days}-day steps of the same workload with {all_threads} threads "
                      f"({wn:.1f} s) and {s1} with one ({w1:.1f} s), its "
                      f"{len(case.report_dt)}-step schedule repeated from the initial state; "
                      f"the oracle's C built with -O3 -march=native, OpenMP assembly and "
                      f"Jacobian product, serial ILU(0) and BiCGStab"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed report steps (default: 30 for c2, 10 for c3, 20 for c4)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c3-mixed", "c4-ensemble", "c5", "c5-guess", "c5-kernels",
                             "c6-live", "c6-wet"],
                    help="c2: the headline metric line; c5: the same line on the 500k-cell "
                         "waterflood (100x100x50); c6-live: the same line on a 24x25x15 "
                         "live-oil depletion with phase appearance; c3-mixed: FP32 ILU(0) vs FP64 on the "
                         "masked 45k-cell grid; c4-ensemble: 64 members in one launch; "
                         "c5-guess: learned Newton guess on the 500k-cell waterflood; "
                         "c5-kernels: per-kernel HBM roofline at 500k cells")
    ap.add_argument("--train-seeds", type=int, default=8, help="training seeds (c5-guess)")
    ap.add_argument("--test-seeds", type=int, default=2, help="held-out seeds (c5-guess)")
    ap.add_argument("--epochs", type=int, default=100, help="training epochs (c5-guess)")
    ap.add_argument("--lr", type=float, default=3e-3, help="Adam step size (c5-guess)")
    ap.add_argument("--save-net", default=None, help="save the trained parameters (.npy)")
    ap.add_argument("--members", type=int, default=64, help="ensemble size (c4-ensemble)")
    ap.add_argument("--member-split", default="6x6",
                    help="c4-ensemble: AxB whole-column subdomains of a block ILU0 in every member "
                         "(none: each member's ILU(0) of the whole system, one workgroup each)")
    ap.add_argument("--one-wg-steps", type=int, default=5,
                    help="c4-ensemble: report steps of the one-workgroup-per-member reference run "
                         "(0: none)")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of autotuned ensemble launch shapes (c4-ensemble)")
    ap.add_argument("--baseline-members", type=int, default=4,
                    help="members timed one by one on the single-system FP64 path (c4-ensemble)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 FP32 ILU(0) factors")
    ap.add_argument("--ilu-blocks", default="4x4",
                    help="block ILU0 subdomain boxes: 'BXxBY' columns over the full depth, "
                         "'BXxBYxBZ', or 'none' for the single-block ILU(0) (c2, c3-mixed, "
                         "c5-guess, and the block rows of c5-kernels)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="time budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--krylov-graph", type=int, default=1,
                    help="replay BiCGStab chunks from HIP graphs (1) or enqueue kernel by kernel (0)")
    ap.add_argument("--krylov", choices=["bicgstab", "gmres"], default="bicgstab",
                    help="Newton's linear solver (c2)")
    ap.add_argument("--restart", type=int, default=30, help="GMRes restart length")
    ap.add_argument("--precond", choices=["ilu0", "cpr"], default="ilu0",
                    help="Newton's preconditioner: the (block-)ILU(0), or CPR-AMG with it as "
                         "the second stage")
    ap.add_argument("--wells", choices=["simplified", "standard"], default="simplified",
                    help="c2 / c6-live: fixed-source wells, or standard wells with their own "
                         "unknowns solved by the Schur complement")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--kernel-grid", default="100x100x50",
                    help="grid of the c5-kernels table (C5: 100x100x50; 200x200x50 is the 2M-cell "
                         "stand-in)")
    ap.add_argument("--kernels", default=None,
                    help="comma-separated subset of the c5-kernels table (spmv, ilu0_apply_fp64, "
                         "ilu0_apply_fp32, assemble, ilu0_factor_fp64)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (a reference "
                         "kernel for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path is single-GPU; --gpus {args.gpus} "
              "is not supported)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_06059_amd import cases, opm

    torch.cuda.set_device(0)
    opm.init()
    opm.set_option(opm.OPT_KRYLOV_GRAPH, args.krylov_graph)
    if args.workload == "c3-mixed":
        return bench_mixed(args)
    if args.workload == "c4-ensemble":
        return bench_ensemble(args)
    if args.workload == "c5-guess":
        return bench_guess(args)
    if args.workload == "c5-kernels":
        return bench_kernels(args)
    if args.steps is None:
        args.steps = 30
    live = args.workload in ("c6-live", "c6-wet")
    if args.workload == "c6-wet":
        case = cases.config_wet()
        workload = ("12x12x5 wet-gas case: dry gas (2 MMscf/d) into undersaturated oil whose gas "
                    "vaporises up to r_v = 0.01 sm3/sm3 at 3000 psi, 720 cells, 30-day steps")
    elif args.workload == "c5":
        case = cases.config5(seed=5008)
        workload = ("100x100x50 waterflood, 500000 cells (4 injectors, 5 producers), 10-day "
                    "implicit steps")
    elif live:
        case = cases.config_live(nx=24, ny=25, nz=15)
        workload = ("24x25x15 live-oil depletion (bubble point 3000 psi, producer at 2500 psi: "
                    "free gas appears), 9000 cells, 15-day implicit steps")
    else:
        case = cases.config2()
        workload = "24x25x15 waterflood, 9000 cells, 10-day implicit steps"
    if args.wells == "standard":
        case.standard_wells = True
    opts = opm.default_opts(case, precision=args.precision)
    if args.krylov == "gmres":
        opts.krylov, opts.restart = opm.KRYLOV_GMRES, args.restart
    if args.precond == "cpr":
        opts.precond = opm.PRECOND_CPR
    dt = case.report_dt[0]
    stream = torch.cuda.current_stream()
    blocks = parse_blocks(args.ilu_blocks, case)

    def run(blk):
        """Warm-up steps, then the timed report steps from the state they
        leave (inputs resident in HBM)."""
        g = opm.GpuModel(case, device="cuda:0", ilu_blocks=blk)
        y = g.initial_state()
        for _ in range(args.warmup):
            st, rep = g.advance(y, dt, opts)
            if st != opm.OK:
                raise RuntimeError(f"warm-up step failed: {opm._strerror(st)}")
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st, rep = g.advance(y, dt, opts)
            if st != opm.OK:
                raise RuntimeError(f"timed step failed: {opm._strerror(st)}")
            reps.append(rep.as_dict())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return g, y, reps, wall

    g, y, reps, wall = run(blocks)
    cni = sum(r["cell_newton_its"] for r in reps)
    newton = sum(r["newton_its"] for r in reps)
    lin = sum(r["lin_its"] for r in reps)
    value = cni / wall
    other = None
    if blocks is not None:   # the single-block ILU(0) on the same workload
        g1, y1, reps1, wall1 = run(None)
        c1 = sum(r["cell_newton_its"] for r in reps1)
        n1 = sum(r["newton_its"] for r in reps1)
        l1 = sum(r["lin_its"] for r in reps1)
        yb, ys = y.cpu().numpy(), y1.cpu().numpy()
        other = {"value": round(c1 / wall1, 1), "ms_per_step": round(1e3 * wall1 / args.steps, 3),
                 "newton_its": n1, "lin_its_per_newton": round(l1 / max(n1, 1), 2),
                 "preconditioner": "ILU(0) of the whole system (sec. 2.3.1), one workgroup "
                                   f"walking its {g1.n_levels} hyperplane levels",
                 "final_state_vs_block": {
                     "p_rel": float(abs(yb[:, 0] - ys[:, 0]).max() / abs(ys[:, 0]).max()),
                     "s_abs": float(abs(yb[:, 1:] - ys[:, 1:]).max())},
                 "speedup_of_block": round(value / (c1 / wall1), 3)}
        del g1, y1

    # ---- dominant kernel: HIP-event timing of repeated launches ------------
    acc0 = g.accumulation(y)
    yk = y.clone()
    yk[:, 0] += 1e4   # a state off equilibrium: a representative system
    R, J, _ = g.assemble(yk, acc0, dt)
    ilu, status = g.ilu0_factor(J, args.precision)
    r = R.clone()
    x = g.zeros_state()
    L = opm.lib()
    pbp = g._pbp()
    sp = opm._ptr
    s = opm._stream()

    def timed(fn, reps):
        for _ in range(5):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    if args.copy_probe_mb > 0:
        nbytes = args.copy_probe_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=g.dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t_apply = timed(lambda: L.opm_ilu0_apply(pbp, sp(ilu), args.precision, sp(r), sp(x), s),
                    args.kernel_reps)
    t_spmv = timed(lambda: L.opm_spmv(pbp, sp(J), sp(r), sp(x), s), args.kernel_reps)
    norms = torch.zeros(L.opm_norms_bytes(pbp) // 8, dtype=torch.float64, device=g.dev)
    Rb = torch.empty_like(R)
    Jb = torch.empty_like(J)
    t_asm = timed(lambda: L.opm_assemble(pbp, sp(yk), sp(acc0), dt, sp(Rb), sp(Jb), sp(norms), s),
                  args.kernel_reps)
    n = g.n
    spmv_b = spmv_bytes_per_cell(g.nnzb, n) * n
    asm_b = assemble_bytes(n, g.nnzb, g.nf)
    if blocks is not None:
        apply_class = "block_apply"
        apply = {"seconds": t_apply, "bytes": block_sweep_bytes_per_cell(args.precision) * n,
                 "kernel": f"block-ILU0 forward+backward sweeps (k_apply_blocks, one 64-thread "
                           f"workgroup per subdomain, {g.pb.n_sub} subdomains)"}
    else:
        apply_class = "ilu0_apply"
        apply = {"seconds": t_apply, "bytes": sweep_bytes_per_cell(args.precision) * n,
                 "kernel": "ilu0 forward+backward sweeps (k_gather_rhs + k_apply_ring2, "
                           "one workgroup of 512 threads)"}
    kernels = {
        apply_class: apply,
        "spmv": {"seconds": t_spmv, "bytes": spmv_b, "kernel": "k_spmv"},
        "assemble": {"seconds": t_asm, "bytes": asm_b, "kernel": "k_assemble_tiled+k_norms_final"},
    }
    # time share of each kernel class in one Newton iteration of the run
    its_per_newton = lin / max(newton, 1)
    share = {apply_class: 2 * its_per_newton * t_apply, "spmv": 2 * its_per_newton * t_spmv,
             "assemble": t_asm}
    dom = max(share, key=share.get)
    k = kernels[dom]
    achieved = k["bytes"] / k["seconds"] / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(dom, args.precision) if args.workload == "c2" else None,
                "kernel": k["kernel"], "avg_launch_us": round(k["seconds"] * 1e6, 3),
                "bytes_per_launch": int(k["bytes"])}

    if blocks is not None:
        precond = (f"block ILU0 (sec. 2.5, one block per subdomain): {g.pb.n_sub} column "
                   f"subdomains of {blocks[0]}x{blocks[1]}x{blocks[2]} cells")
    else:
        precond = "ILU(0) of the whole system (sec. 2.3.1)"
    if args.precond == "cpr":
        lv = g.amg_levels()
        precond = (f"CPR-AMG (sec. 2.3.1): quasi-IMPES pressure system, one V(1,1) cycle of a "
                   f"{len(lv)}-level aggregation AMG (unknowns per level "
                   f"{'/'.join(str(a) for a, _ in lv)}), then as the second stage " + precond)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "cell-Newton-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64+f32-ilu",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n_cells": n, "nnzb": g.nnzb, "ilu_levels": g.n_levels,
                   "newton_tol_cnv": case.tol_cnv, "lin_rtol": case.lin_rtol,
                   "precision": "fp64" if args.precision == 0 else "mixed",
                   "krylov": "BiCGStab" if args.krylov == "bicgstab" else f"GMRes({args.restart})",
                   "wells": ("standard wells (Q_t, F_w, F_g, p_bhp per well; Schur complement)"
                             if args.wells == "standard" else "fixed sources / BHP sinks"),
                   "preconditioner": precond},
        "roofline": roofline,
        "breakdown": {
            "newton_its": newton, "lin_its_per_newton": round(its_per_newton, 2),
            "t_assemble_s": round(sum(r["t_assemble"] for r in reps), 4),
            "t_factor_s": round(sum(r["t_factor"] for r in reps), 4),
            "t_krylov_s": round(sum(r["t_krylov"] for r in reps), 4),
            "t_update_s": round(sum(r["t_update"] for r in reps), 4),
            "kernels_us": {kk: round(v["seconds"] * 1e6, 2) for kk, v in kernels.items()},
            "kernels_gbs": {kk: round(v["bytes"] / v["seconds"] / 1e9, 1) for kk, v in kernels.items()},
        },
    }
    if other is not None:
        line["single_block_ilu0"] = other
    if live:
        line["live_oil"] = {"free_gas_cells_at_end": int((g.meaning() == 0).sum()),
                            "oil_free_cells_at_end": int((g.meaning() == 2).sum()), "n_cells": n}

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(case, dt, opts, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
