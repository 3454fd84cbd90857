"""Writes couette_step_oracle.json: one SSP-RK3 step (dt = 1e-3, no
projection) of the full Couette workload by the oracle (two species, N = 32,
icosahedron M = 12, N_rho = 16, K = 16 elements of degree 3, 64 nodes,
diffuse walls), reduced to what a GPU test can compare.  With
dF = F(t + dt) - F(t):

  * a fingerprint of the seeded input (so the test knows it runs the same F);
  * max |dF| over the whole state (the scale of the bar);
  * at eight nodes (both walls, element boundaries, the middle) and both
    species: dF at 48 fixed sampled points, at 16 points drawn among those
    with |dF| >= 1% of that array's max, and at its max;
  * four projections sum W_k dF of the whole increment onto seeded normal
    weights, which see an error anywhere.

With --nyquist it writes couette_step_nyquist_oracle.json: the same step
under the Nyquist-zeroed variant of the gain (the plan option nyquist_zero).
With --projected it writes couette_step_projected_oracle.json instead: the
same step with each node's collision term projected onto the conserved
moments (the FP32-mixed leg of the benchmark), plus the loss scale
Lambda = max over the stored nodes and species p of sum_q max |loss^{pq}| at
the initial state, from which the FP32-mixed bar is stated.

The step takes 768 collision evaluations (3 stages x 64 nodes x 4 ordered
pairs), about 28 minutes on 8 host cores.
Only the oracle is called (the input comes from the seeded workload
generator).

    python tests/golden/make_couette_step_oracle.py [--projected | --nyquist]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SAMPLE_SEED, PROJ_SEED, N_SAMPLES, N_BULK, N_PROJ = 31337, 4242, 48, 16, 4
NODES = [0, 1, 3, 4, 21, 32, 62, 63]


def main():
    import argparse
    import numpy as np
    from oracle import conservation as cons
    from oracle import dg as odg
    from oracle.collide import PairPlan, collide_gain_loss, mixture_collision
    ap = argparse.ArgumentParser()
    grp = ap.add_mutually_exclusive_group()
    grp.add_argument("--projected", action="store_true")
    grp.add_argument("--nyquist", action="store_true")
    args = ap.parse_args()
    projected, nyquist = args.projected, args.nyquist
    from oracle.quadrature import sphere_set
    from paper_1903_04670_amd import workloads as wl
    cfg = wl.couette_two_species()
    F0 = cfg["F"]
    ns = cfg["ns"]
    s, w = sphere_set(cfg["sphere"], cfg["M"])
    opl = [[PairPlan(cfg["N"], cfg["L"], cfg["masses"][p], cfg["masses"][q], cfg["omega"][p][q],
                     cfg["alpha"][p][q], cfg["Nrho"], s, w, R=cfg["R"][p][q], nyquist_zero=nyquist)
            for q in range(ns)]
           for p in range(ns)]
    prob = odg.Couette1D(cfg["N"], cfg["L"], cfg["masses"], cfg["K"], cfg["P"], cfg["u_left"], cfg["u_right"])
    stage = [0]

    def coll(Y):
        C = mixture_collision(opl, Y)
        if projected:
            C = np.stack([cons.project(C[i], cfg["N"], cfg["L"], cfg["masses"]) for i in range(C.shape[0])])
        return C

    def rhs(X):
        stage[0] += 1
        print("stage %d" % stage[0], flush=True)
        return prob.rhs(X, coll)
    F1 = odg.ssp_rk3(F0, cfg["dt"], rhs)
    dF = F1 - F0
    n3 = cfg["N"] ** 3
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(n3, N_SAMPLES, replace=False))
    nodes = []
    for i in NODES:
        per = []
        for p in range(ns):
            d = dF[i, p].ravel()
            am = int(np.argmax(np.abs(d)))
            bulk = np.flatnonzero(np.abs(d) >= 0.01 * np.abs(d[am]))
            bidx = np.sort(np.random.default_rng(SAMPLE_SEED + 1 + 2 * i + p).choice(bulk, N_BULK, replace=False))
            per.append(dict(amax=float(np.abs(d[am])), argmax=am, at_argmax=float(d[am]),
                            samples=[float(v) for v in d[idx]], bulk_idx=[int(v) for v in bidx],
                            bulk=[float(v) for v in d[bidx]]))
        nodes.append(dict(node=i, species=per))
    W = np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, dF.size))
    lam = None
    if projected:
        lam = 0.0
        # over the stored nodes (the nodes' inputs differ by 1% noise, and a
        # smaller scale only tightens the bar)
        for i in NODES:
            for p in range(ns):
                lam = max(lam, sum(float(np.max(np.abs(collide_gain_loss(opl[p][q], F0[i, p], F0[i, q])[1])))
                                   for q in range(ns)))
    doc = dict(workload=cfg["name"], dt=cfg["dt"], projection=projected, nyquist_zero=nyquist, loss_scale=lam,
               sample_seed=SAMPLE_SEED,
               proj_seed=PROJ_SEED, n_proj=N_PROJ, sample_idx=[int(v) for v in idx],
               inputs=dict(shape=list(F0.shape), total=float(F0.sum()),
                           sums=[[float(F0[i, p].sum()) for p in range(ns)] for i in NODES]),
               dmax=float(np.max(np.abs(dF))), proj=[float(v) for v in W @ dF.ravel()],
               nodes=nodes)
    name = ("couette_step_projected_oracle.json" if projected else
            "couette_step_nyquist_oracle.json" if nyquist else "couette_step_oracle.json")
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    print("written; max |dF| %.6e" % doc["dmax"])


if __name__ == "__main__":
    main()
