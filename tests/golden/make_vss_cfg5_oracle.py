"""Writes vss_cfg5_oracle.json: the oracle's collision terms of the VSS
precision workload at its full shape (three species, masses 1, 2, 4,
alpha = 1.4, N = 48, Fibonacci M = 32, N_rho = 24), for all nine ordered
pairs at two nodes, reduced to what a GPU test can compare:

  * a fingerprint of the seeded input (so the test knows it runs the same F);
  * max |Q| and max |loss| (the scales of the FP64 and FP32-mixed bars);
  * Q at 96 fixed sampled points (most of them in the tails), at 32 points
    drawn among those with |Q| >= 1% of max |Q| (per node), and at the point
    of max |Q|;
  * four projections sum_v W_k(v) Q(v) onto seeded normal weights, which
    see an error anywhere (sum_v |W_k(v) Q(v)| is kept beside them).

The full terms (110,592 values each) are too large to keep, and the oracle
needs about 3 minutes per pair for the gain table and 20 s per evaluation on
8 cores, too slow for a test.  Only the oracle is called (the input comes
from the seeded workload generator).

    python tests/golden/make_vss_cfg5_oracle.py [-j 4]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE_SEED, PROJ_SEED, N_SAMPLES, N_BULK, N_PROJ = 20260, 777, 96, 32, 4
NODES = 2


def _one(pq):
    import numpy as np
    from oracle.collide import PairPlan, collide_gain_loss
    from oracle.quadrature import sphere_set
    from paper_1903_04670_amd import workloads as wl
    p, q = pq
    cfg = wl.precision_vss(n_nodes=NODES)
    s, w = sphere_set(cfg["sphere"], cfg["M"])
    plan = PairPlan(cfg["N"], cfg["L"], cfg["masses"][p], cfg["masses"][q], cfg["omega"][p][q],
                    cfg["alpha"][p][q], cfg["Nrho"], s, w, R=cfg["R"][p][q])
    n3 = cfg["N"] ** 3
    idx = sample_indices(n3)
    W = projection_weights(n3)
    out = []
    for i in range(NODES):
        gain, loss = collide_gain_loss(plan, cfg["F"][i, p], cfg["F"][i, q])
        Q = (gain - loss).ravel()
        if not np.all(np.isfinite(Q)):
            raise RuntimeError("non-finite oracle output for pair %s node %d" % (pq, i))
        am = int(np.argmax(np.abs(Q)))
        bulk = np.flatnonzero(np.abs(Q) >= 0.01 * np.abs(Q[am]))
        bidx = np.sort(np.random.default_rng(SAMPLE_SEED + 1 + i).choice(bulk, min(N_BULK, bulk.size), replace=False))
        out.append(dict(qmax=float(np.max(np.abs(Q))), lossmax=float(np.max(np.abs(loss))),
                        argmax=am, at_argmax=float(Q[am]), samples=[float(v) for v in Q[idx]],
                        bulk_idx=[int(v) for v in bidx], bulk=[float(v) for v in Q[bidx]],
                        proj=[float(v) for v in W @ Q], proj_scale=[float(v) for v in np.abs(W) @ np.abs(Q)]))
        print("pair (%d,%d) node %d: max|Q| %.6e" % (p, q, i, out[-1]["qmax"]), flush=True)
    return "%d,%d" % pq, out


def sample_indices(n3):
    import numpy as np
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n3, N_SAMPLES, replace=False))


def projection_weights(n3):
    import numpy as np
    return np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, n3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=4)
    args = ap.parse_args()
    # split the cores between the workers before numpy starts its threads
    os.environ.setdefault("OMP_NUM_THREADS", str(max(1, (os.cpu_count() or 1) // args.j)))
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    from paper_1903_04670_amd import workloads as wl
    cfg = wl.precision_vss(n_nodes=NODES)
    F = cfg["F"]
    inputs = dict(shape=list(F.shape), sums=[[float(F[i, p].sum()) for p in range(cfg["ns"])] for i in range(NODES)],
                  first=[[float(F[i, p].flat[0]) for p in range(cfg["ns"])] for i in range(NODES)])
    pairs = [(p, q) for p in range(cfg["ns"]) for q in range(cfg["ns"])]
    with ProcessPoolExecutor(args.j) as ex:
        res = dict(ex.map(_one, pairs))
    doc = dict(workload=cfg["name"], nodes=NODES, sample_seed=SAMPLE_SEED, proj_seed=PROJ_SEED,
               n_samples=N_SAMPLES, n_proj=N_PROJ, inputs=inputs,
               sample_idx=[int(v) for v in sample_indices(cfg["N"] ** 3)],
               pairs={k: res[k] for k in sorted(res)})
    with open(os.path.join(HERE, "vss_cfg5_oracle.json"), "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    print("written", np.sum([len(v) for v in res.values()]), "evaluations")


if __name__ == "__main__":
    main()
