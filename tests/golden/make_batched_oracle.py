"""Writes batched_oracle.json: the oracle's collision terms for 32 of the
1024 instances of the batching workload (every 32nd; N in {16, 24, 32},
1-3 species, N_rho in {8, 16}), all their ordered pairs, reduced to what a
GPU test can compare: per (instance, pair) max |Q|, Q at 32 fixed sampled
points and at its max, and two projections of the whole term onto seeded
normal weights, with the sum of each instance's input as its fingerprint.

135 evaluations, a few minutes on 8 host cores.  Only the oracle is called
(the input comes from the seeded workload generator).

    python tests/golden/make_batched_oracle.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

N_INST, STRIDE, SAMPLE_SEED, PROJ_SEED, N_SAMPLES, N_PROJ = 1024, 32, 5151, 6262, 32, 2


def sample_indices(N):
    import numpy as np
    return np.sort(np.random.default_rng(SAMPLE_SEED + N).choice(N ** 3, N_SAMPLES, replace=False))


def projection_weights(N):
    import numpy as np
    return np.random.default_rng(PROJ_SEED + N).standard_normal((N_PROJ, N ** 3))


def main():
    import numpy as np
    from oracle.collide import PairPlan, collide
    from oracle.quadrature import sphere_set
    from paper_1903_04670_amd import workloads as wl
    insts = wl.batched_instances(n_inst=N_INST)
    out = {}
    for k in range(0, N_INST, STRIDE):
        cfg = insts[k]
        N, ns = cfg["N"], cfg["ns"]
        s, w = sphere_set(cfg["sphere"], cfg["M"])
        idx, W = sample_indices(N), projection_weights(N)
        pairs = {}
        for p in range(ns):
            for q in range(ns):
                plan = PairPlan(N, cfg["L"], cfg["masses"][p], cfg["masses"][q], cfg["omega"][p][q],
                                cfg["alpha"][p][q], cfg["Nrho"], s, w, R=cfg["R"][p][q])
                nodes = []
                for i in range(cfg["n_nodes"]):
                    Q = collide(plan, cfg["F"][i, p], cfg["F"][i, q]).ravel()
                    am = int(np.argmax(np.abs(Q)))
                    nodes.append(dict(qmax=float(np.abs(Q[am])), argmax=am, at_argmax=float(Q[am]),
                                      samples=[float(v) for v in Q[idx]], proj=[float(v) for v in W @ Q]))
                pairs["%d,%d" % (p, q)] = nodes
        out[str(k)] = dict(N=N, ns=ns, Nrho=cfg["Nrho"], fsum=float(cfg["F"].sum()), pairs=pairs)
        print("instance %d: N=%d ns=%d N_rho=%d" % (k, N, ns, cfg["Nrho"]), flush=True)
    doc = dict(workload="batched_instances(n_inst=%d)" % N_INST, stride=STRIDE, sample_seed=SAMPLE_SEED,
               proj_seed=PROJ_SEED, n_samples=N_SAMPLES, n_proj=N_PROJ, instances=out)
    with open(os.path.join(HERE, "batched_oracle.json"), "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    print("written", len(out), "instances")


if __name__ == "__main__":
    main()
