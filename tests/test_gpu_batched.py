"""Heterogeneous batched launch: items of different N, species counts and
quadratures in one launch per stage, bit-identical to one dgfs_collide call
per item, and equal to the oracle on sampled items."""
import numpy as np
import pytest

from helpers import gpu_plan, oracle_pairs, rel_linf, small_config
from oracle.collide import collide as oracle_collide
from paper_1903_04670_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, insts, precision):
    from paper_1903_04670_amd import dgfs
    plans, items, outs_b, outs_s, tensors = [], [], [], [], []
    for k, cfg in enumerate(insts):
        pl = gpu_plan(cfg, precision=precision, nyquist_zero=cfg.get("nyquist_zero", False))
        plans.append(pl)
        F = torch.from_numpy(cfg["F"]).cuda()
        tensors.append(F)
        for p in range(cfg["ns"]):
            for q in range(cfg["ns"]):
                ob = torch.zeros(F[:, p].shape, dtype=torch.float64, device="cuda")
                items.append((k, p, q, F[:, p], F[:, q], ob))
                outs_b.append(ob)
                outs_s.append(dgfs.collide(pl, p, q, F[:, p], F[:, q]))
    dgfs.collide_batched(plans, items)
    torch.cuda.synchronize()
    return plans, items, outs_b, outs_s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_small_mixed_sizes(torch_cuda, precision):
    """N in {8, 12, 16}, 1-3 species, several nodes per item, one VSS
    instance among VHS ones."""
    torch = torch_cuda
    insts = []
    rng = np.random.default_rng(8)
    for i in range(9):
        N = [8, 12, 16][i % 3]
        cfg = small_config(N, ns=1 + i % 3, Nrho=int(rng.choice([3, 4])), seed=40 + i, n_nodes=1 + i % 2,
                           M_kind=["icosahedron", "octahedron", "fibonacci"][i % 3])
        if i == 4:
            cfg["alpha"] = np.full((cfg["ns"], cfg["ns"]), 1.4)
        insts.append(cfg)
    plans, items, outs_b, outs_s = _run(torch, insts, precision)
    for ob, os_ in zip(outs_b, outs_s):
        assert torch.equal(ob, os_)
    if precision == "fp64":
        for (k, p, q, _, _, ob) in items[::3]:
            cfg = insts[k]
            opl = oracle_pairs(cfg)
            got = ob.cpu().numpy()
            for i in range(cfg["n_nodes"]):
                ref = oracle_collide(opl[p][q], cfg["F"][i, p], cfg["F"][i, q])
                assert rel_linf(got[i], ref) <= 1e-11


def _check_stored_oracle(insts, items):
    """Every 32nd instance of the 1024, all its ordered pairs, against the
    oracle terms stored by tests/golden/make_batched_oracle.py: 32 sampled
    points and the point of max |Q| within 1e-11 of max |Q|, and two
    projections of the whole term within 1e-11 max |Q| ||W||_2."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "batched_oracle.json")) as fh:
        gold = json.load(fh)
    by_item = {(k, p, q): ob for (k, p, q, _, _, ob) in items}
    checked, worst = 0, 0.0
    for ks, g in gold["instances"].items():
        k = int(ks)
        cfg = insts[k]
        assert (cfg["N"], cfg["ns"], cfg["Nrho"]) == (g["N"], g["ns"], g["Nrho"])
        assert abs(cfg["F"].sum() - g["fsum"]) <= 1e-12 * abs(g["fsum"])
        N = cfg["N"]
        idx = np.sort(np.random.default_rng(gold["sample_seed"] + N).choice(N ** 3, gold["n_samples"], replace=False))
        W = np.random.default_rng(gold["proj_seed"] + N).standard_normal((gold["n_proj"], N ** 3))
        wn = np.linalg.norm(W, axis=1)
        for key, nodes in g["pairs"].items():
            p, q = map(int, key.split(","))
            got = by_item[(k, p, q)].cpu().numpy().reshape(cfg["n_nodes"], -1)
            for i, r in enumerate(nodes):
                Q = got[i]
                e = max(float(np.max(np.abs(Q[idx] - np.asarray(r["samples"])))), abs(Q[r["argmax"]] - r["at_argmax"]))
                ep = float(np.max(np.abs(W @ Q - np.asarray(r["proj"])) / wn))
                worst = max(worst, e / r["qmax"], ep / r["qmax"])
                assert e <= 1e-11 * r["qmax"] and ep <= 1e-11 * r["qmax"], (k, p, q, i)
                checked += 1
    assert checked == sum(insts[int(k)]["ns"] ** 2 * insts[int(k)]["n_nodes"] for k in gold["instances"])
    print("stored oracle: %d instances, %d terms, worst %.3e of max|Q|" % (len(gold["instances"]), checked, worst))


@pytest.mark.parametrize("n_inst,precision", [(96, "fp64"), (1024, "fp64"), (1024, "fp32")])
def test_batched_uneven_instances_N16_24_32(torch_cuda, n_inst, precision):
    """Space-homogeneous instances drawn like the batching workload (N in
    {16, 24, 32}, 1-3 species, N_rho in {8, 16}, icosahedron), 96 of them
    and the workload's full 1024 in the launch configuration the benchmark
    times: the batched launch equals per-instance launches bit for bit; in
    the 96-instance case 16 instances with N <= 24 (all their ordered
    pairs) and one pair of an N = 32 instance are checked against the
    oracle.  The FP32-mixed plans run the same 1024 instances, also bit for
    bit against their per-instance launches.  In FP64, every 32nd of the
    1024 instances (all ordered pairs) is checked against stored oracle
    terms."""
    torch = torch_cuda
    insts = wl.batched_instances(n_inst=n_inst)
    plans, items, outs_b, outs_s = _run(torch, insts, precision)
    assert len(items) > n_inst
    for ob, os_ in zip(outs_b, outs_s):
        assert torch.equal(ob, os_)
    if n_inst == 1024 and precision == "fp64":
        _check_stored_oracle(insts, items)
    if n_inst > 96:
        return
    # sampled instances against the oracle
    small = [k for k, cfg in enumerate(insts) if cfg["N"] <= 24][:16]
    big = [k for k, cfg in enumerate(insts) if cfg["N"] == 32][:1]
    checked = 0
    done_big = set()
    opl_cache = {}
    for (k, p, q, _, _, ob) in items:
        if k in big:
            if k in done_big:
                continue
            done_big.add(k)
        if k in small or k in big:
            cfg = insts[k]
            if k not in opl_cache:
                opl_cache[k] = oracle_pairs(cfg)
            got = ob.cpu().numpy()
            for i in range(cfg["n_nodes"]):
                ref = oracle_collide(opl_cache[k][p][q], cfg["F"][i, p], cfg["F"][i, q])
                assert rel_linf(got[i], ref) <= 1e-11, (k, p, q, i)
            checked += 1
    assert checked >= 17


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_radix5_radix7_grids_equal_single_calls(torch_cuda, precision):
    """Items on N = 10, 14, 40, 56 (radix-5 and radix-7 transforms) with an
    N = 16 item in one batched launch per stage (the N <= 56 class): bit for
    bit the single-plan results; the N = 40 item against the oracle."""
    torch = torch_cuda
    insts = []
    for k, (N, ns) in enumerate([(10, 2), (14, 1), (16, 2), (40, 1), (56, 1)]):
        insts.append(small_config(N, ns=ns, Nrho=2, seed=90 + k, n_nodes=1,
                                  M_kind="octahedron" if N >= 40 else "icosahedron"))
    plans, items, outs_b, outs_s = _run(torch, insts, precision)
    for ob, os_ in zip(outs_b, outs_s):
        assert torch.equal(ob, os_)
    if precision == "fp64":
        cfg = insts[3]
        ref = oracle_collide(oracle_pairs(cfg)[0][0], cfg["F"][0, 0], cfg["F"][0, 0])
        got = [ob for (k, p, q, _, _, ob) in items if k == 3][0].cpu().numpy()[0]
        assert rel_linf(got, ref) <= 1e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_one_group_blocks_vss_and_packed_equal_single_calls(torch_cuda, precision):
    """Above N = 32 a gain block is one group of 2N lanes, and the batched
    launch's 128-thread blocks carry lanes outside it: a VSS item (alpha =
    1.3, Fibonacci M = 7) and a Nyquist-zeroed item on N = 40, with an N = 12
    item, in one batched launch per stage give bit for bit the single-plan
    results."""
    torch = torch_cuda
    vss = small_config(40, ns=1, M_kind="fibonacci", Nrho=2, seed=95, n_nodes=1)
    vss["alpha"] = np.full((1, 1), 1.3)
    nyq = small_config(40, ns=2, M_kind="octahedron", Nrho=2, seed=96, n_nodes=1)
    nyq["nyquist_zero"] = True
    insts = [small_config(12, ns=1, Nrho=3, seed=97, n_nodes=2), vss, nyq]
    plans, items, outs_b, outs_s = _run(torch, insts, precision)
    for ob, os_ in zip(outs_b, outs_s):
        assert torch.equal(ob, os_)


def test_batched_accumulate_empty_items_and_strided_outputs(torch_cuda):
    """DGFS_ACCUMULATE on a batch equals one accumulating dgfs_collide per
    item bit for bit; items with zero nodes are skipped (alone, a batch of
    them is a no-op); outputs may be node-strided views of a species-major
    array."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    rng = np.random.default_rng(21)
    insts = [small_config(8, ns=2, Nrho=3, seed=61, n_nodes=3),
             small_config(12, ns=1, Nrho=3, seed=62, n_nodes=2, M_kind="octahedron"),
             small_config(16, ns=2, Nrho=2, seed=63, n_nodes=1, M_kind="fibonacci")]
    plans = [gpu_plan(cfg) for cfg in insts]
    items, outs_b, outs_s = [], [], []
    for k, cfg in enumerate(insts):
        F = torch.from_numpy(cfg["F"]).cuda()
        ns, N = cfg["ns"], cfg["N"]
        shape = (cfg["n_nodes"], ns * ns, N, N, N)
        base = torch.from_numpy(rng.standard_normal(shape) * 1e-3).cuda()
        Ob, Os = base.clone(), base.clone()      # out[:, p * ns + q] is node-strided; no two items share one
        for p in range(ns):
            for q in range(ns):
                items.append((k, p, q, F[:, p], F[:, q], Ob[:, p * ns + q]))
                dgfs.collide(plans[k], p, q, F[:, p], F[:, q], out=Os[:, p * ns + q], accumulate=True)
        items.append((k, 0, 0, F[:0, 0], F[:0, 0], Ob[:0, 0]))   # zero nodes
        outs_b.append(Ob)
        outs_s.append(Os)
    dgfs.collide_batched(plans, items, accumulate=True)
    torch.cuda.synchronize()
    for Ob, Os in zip(outs_b, outs_s):
        assert torch.equal(Ob, Os)
    # a batch of empty items leaves everything as it was
    before = [o.clone() for o in outs_b]
    dgfs.collide_batched(plans, [it for it in items if it[3].shape[0] == 0])
    torch.cuda.synchronize()
    for o, b in zip(outs_b, before):
        assert torch.equal(o, b)


def test_prepared_batch_reruns_on_current_inputs(torch_cuda):
    """dgfs.Batch builds its descriptor array once; run() twice, the inputs
    overwritten in place between the runs: each run equals one dgfs_collide
    call per item on the inputs of that time, bit for bit (the descriptors
    hold addresses, not values).  An N = 32 FP64 item runs the half-wave gain
    body, two x-planes per block, in both launches."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    insts = [small_config(8, ns=2, Nrho=3, seed=71, n_nodes=2),
             small_config(32, ns=1, Nrho=2, seed=72, n_nodes=1),
             small_config(16, ns=1, Nrho=3, seed=73, n_nodes=2, M_kind="octahedron")]
    plans = [gpu_plan(cfg) for cfg in insts]
    Fs = [torch.from_numpy(cfg["F"]).cuda() for cfg in insts]
    items = []
    for k, cfg in enumerate(insts):
        for p in range(cfg["ns"]):
            for q in range(cfg["ns"]):
                items.append((k, p, q, Fs[k][:, p], Fs[k][:, q], torch.zeros_like(Fs[k][:, p])))
    batch = dgfs.Batch(plans, items)
    ws = batch.run()
    for rerun in range(2):
        if rerun:
            for F in Fs:
                F.mul_(0.5).add_(F.flip(-1), alpha=0.25)
            batch.run(ws=ws)
        torch.cuda.synchronize()
        for (k, p, q, fp, fq, ob) in items:
            assert torch.equal(ob, dgfs.collide(plans[k], p, q, fp, fq)), (rerun, k, p, q)
