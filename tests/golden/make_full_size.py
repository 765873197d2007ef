"""Write full_size_oracle.json: FP64 oracle results for sampled instances of the
benchmark workloads at their full mesh sizes and time grids.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_full_size.py  (about ten minutes on
eight cores).
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_oracle.json")


def _c1(args):
    level, sample = args
    import workloads as W
    from oracle import timestep
    w = W.mlmc3_mixed_129()
    lv = w.levels[level]
    xi = W.level_xi(w, level, first=sample, n=1)[0]
    qf, _ = timestep.solve_sample(w.problem, xi, lv.steps_per_period, lv.n_periods)
    qc = None
    if lv.coarse_steps_per_period:
        qc, _ = timestep.solve_sample(w.problem, xi, lv.coarse_steps_per_period, lv.n_periods)
    return {"level": level, "sample": sample, "q_fine": float(qf), "q_coarse": None if qc is None else float(qc)}


def _c2(sample):
    import workloads as W
    from oracle import parareal
    w = W.parareal_257()
    pr = w.parareal
    xi = W.level_xi(w, 0, first=sample, n=1)[0]
    res = parareal.run(w.problem, xi, pr.n_periods, pr.n_slices, pr.fine_steps_per_slice,
                       pr.coarse_steps_per_slice, pr.k_max, pr.tol)
    ser = parareal.serial_fine(w.problem, xi, pr.n_periods, pr.n_slices, pr.fine_steps_per_slice)
    return {"sample": sample, "q_parareal": float(res["Q"]), "k": int(res["K"]),
            "jumps": [float(j) for j in res["jumps"]], "q_serial": float(ser["Q"])}


def _c3(sample):
    import workloads as W
    from oracle import picard
    w = W.nonlinear_mlmc4_129()
    lv = w.levels[0]
    xi = W.level_xi(w, 0, first=sample, n=1)[0]
    q, _, counts, flagged = picard.solve_sample(w.problem, xi, lv.steps_per_period, lv.n_periods,
                                                return_counts=True)
    return {"level": 0, "sample": sample, "q": float(q), "picard_iters": int(counts.sum()), "flagged": bool(flagged)}


def _c3_top(sample):
    """A sample of the finest level of the nonlinear workload: fine and coupled coarse run."""
    import workloads as W
    from oracle import picard
    w = W.nonlinear_mlmc4_129()
    level = len(w.levels) - 1
    lv = w.levels[level]
    xi = W.level_xi(w, level, first=sample, n=1)[0]
    qf, _, cf, ff = picard.solve_sample(w.problem, xi, lv.steps_per_period, lv.n_periods, return_counts=True)
    qc, _, cc, fc = picard.solve_sample(w.problem, xi, lv.coarse_steps_per_period, lv.n_periods, return_counts=True)
    return {"level": level, "sample": sample, "q_fine": float(qf), "q_coarse": float(qc),
            "picard_iters_fine": int(cf.sum()), "picard_iters_coarse": int(cc.sum()),
            "flagged": bool(ff or fc)}


def _c4(index):
    import workloads as W
    from oracle import timestep
    r = W.serving_stream(4096)[index]
    prob = W.Problem(r.n_nodes, W.Material(kind=W.MAT_KL))
    q, _ = timestep.solve_sample(prob, list(r.xi), r.steps_per_period, r.n_periods)
    return {"index": index, "n_nodes": r.n_nodes, "steps_per_period": r.steps_per_period,
            "n_periods": r.n_periods, "q": float(q)}


def main():
    import workloads as W
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    # the first 513 x 513 request of the serving stream with the fewest steps
    stream = W.serving_stream(4096)
    big = min((r for r in stream if r.n_nodes == 513), key=lambda r: (r.steps_per_period, r.rid))
    t0 = time.time()
    with ProcessPoolExecutor(8) as ex:
        f1 = [ex.submit(_c1, (l, s)) for l in range(3) for s in (0, 1)]
        f2 = [ex.submit(_c2, 0)]
        f3 = [ex.submit(_c3, s) for s in (0, 1)]
        f4 = [ex.submit(_c4, big.rid)]
        f5 = [ex.submit(_c3_top, 0)]
        out = {"mlmc3_129": [f.result() for f in f1], "parareal_257": [f.result() for f in f2],
               "nonlinear_129": [f.result() for f in f3], "serving": [f.result() for f in f4],
               "nonlinear_129_top": [f.result() for f in f5]}
    out["generator"] = "tests/golden/make_full_size.py (oracle only)"
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
