"""Batched N-way fusion: one persistent launch of many small instances, eager
and replayed from a HIP graph, against the solo launches (bit-exact) and the
CPU oracle (same tolerances as the pair tests)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import hashes as OH
from paper_2007_01277_amd import batch_bench as BB
from paper_2007_01277_amd import hfuse as H

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _init():
    assert torch.cuda.is_available()
    H.hf_init()


def check_instance(kind, x, outs, meta=None):
    xh = x.cpu().numpy()
    if kind in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
        nonce0, tab = meta
        got = outs[0].cpu().numpy().view(np.uint8).reshape(-1, 32)
        hdr = xh.view(np.uint8).tobytes()
        idx = sorted(set([0, 1, len(got) - 1, len(got) // 2]))
        if kind == H.HF_SHA256D:
            ref = OH.sha256d(hdr, nonce0, idx)
        elif kind == H.HF_BLAKE2B:
            ref = OH.blake2b_header(hdr, nonce0, idx)
        else:
            T = tab.cpu().numpy().view(np.uint32)
            ref = [OH.ethash_like_one(hdr, nonce0 + i, T) for i in idx]
        for i, r in zip(idx, ref):
            assert got[i].tobytes() == r, (H.KIND_NAMES[kind], i)
        return
    if kind == H.HF_BN_STATS:
        m_ref, v_ref = oracle.bn_stats(xh)
        m = outs[0].cpu().numpy().astype(np.float64)
        v = outs[1].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(m - m_ref) <= TOL * (np.abs(m_ref) + np.sqrt(v_ref)))
        assert np.all(np.abs(v - v_ref) <= TOL * v_ref)
    elif kind == H.HF_INT_MIX:
        assert np.array_equal(outs[0].cpu().numpy().view(np.uint32), oracle.int_mix(xh.view(np.uint32), 32))
    elif kind == H.HF_IM2COL:
        assert np.array_equal(outs[0].cpu().numpy(), oracle.im2col(xh, 3, 3, 1, 1))
    elif kind == H.HF_LDS_HIST:
        assert np.array_equal(outs[0].cpu().numpy().view(np.uint32).astype(np.uint64), oracle.hist256(xh))
    elif kind == H.HF_MAXPOOL:
        v, i = oracle.maxpool(xh, 3, 3, 2, 1)
        assert np.array_equal(outs[0].cpu().numpy(), v) and np.array_equal(outs[1].cpu().numpy(), i)
    else:
        ref = oracle.upsample(xh, 2)
        mag = oracle.upsample_absmag(xh, 2)
        assert np.all(np.abs(outs[0].cpu().numpy().astype(np.float64) - ref) <= TOL * mag)


def solo_reference(w):
    w.clear()
    for t in w.tasks:
        H.hf_run_solo(t, 256)
    torch.cuda.synchronize()
    return w.snapshot()


def test_batch_matches_solo_and_oracle_every_block():
    kinds, logs, groups = BB.draw(40, seed=11, kmin=8, kmax=14)
    w = BB.Workload(kinds, logs, seed=11)
    ref = solo_reference(w)
    for k, x, o in zip(kinds, w.ins, ref):
        check_instance(k, x, o)
    for block in (256, 512, 1024):
        b = H.Batch(w.tasks, groups, None, block)
        print("batch block", block, b.info(), flush=True)
        w.clear()
        b.run(False)
        torch.cuda.synchronize()
        assert BB.same(ref, w.snapshot()), block
        b.close()


def test_batch_explicit_waves_and_single_member_groups():
    kinds, logs, _ = BB.draw(12, seed=12, kmin=9, kmax=13)
    w = BB.Workload(kinds, logs, seed=12)
    ref = solo_reference(w)
    groups = list(range(12))  # every instance alone
    b = H.Batch(w.tasks, groups, [1] * 12, 512)  # one wavefront each, 7 idle
    w.clear()
    b.run(False)
    torch.cuda.synchronize()
    assert BB.same(ref, w.snapshot())
    b.close()
    groups = [i // 4 for i in range(12)]
    b = H.Batch(w.tasks, groups, [1, 2, 3, 2] * 3, 512)
    w.clear()
    b.run(False)
    torch.cuda.synchronize()
    assert BB.same(ref, w.snapshot())
    b.close()


def test_batch_graph_replays_match_eager():
    kinds, logs, groups = BB.draw(60, seed=13, kmin=10, kmax=15)
    w = BB.Workload(kinds, logs, seed=13)
    ref = solo_reference(w)
    b = H.Batch(w.tasks, groups, None, 256)
    for r in range(4):
        w.clear()
        b.run(True)
        torch.cuda.synchronize()
        assert BB.same(ref, w.snapshot()), f"replay {r}"
        # eager work of the program between replays
        for t in w.tasks[:5]:
            H.hf_run_solo(t, 512)
        torch.cuda.synchronize()
        b.run(False)
        torch.cuda.synchronize()
        assert BB.same(ref, w.snapshot()), f"eager after replay {r}"
    b.close()


def test_batch_worker_intervals_match_solo_every_schedule():
    """Worker-interval schedules: every block x interval size x item size the
    batch admits, eager and replayed from a graph with eager work between the
    replays, bit-exact with the solo launches (checked against the oracle)."""
    kinds, logs, groups = BB.draw(48, seed=15, kmin=8, kmax=15)
    w = BB.Workload(kinds, logs, seed=15)
    ref = solo_reference(w)
    for k, x, o in zip(kinds, w.ins, ref):
        check_instance(k, x, o)
    ran = 0
    for block in (256, 512, 1024):
        for iw in (1, 2, 4, 8):
            if iw > block // 64:
                continue
            for kb in (16, 256):
                sc = H.hf_batch_schedule(block, iw, kb, 0)
                try:
                    b = H.Batch(w.tasks, groups, schedule=sc)
                except H.HFError as e:  # a schedule whose LDS does not fit a CU
                    assert e.status == H.HF_EUNSUPPORTED, (block, iw)
                    continue
                print("workers", block, iw, kb, b.info(), flush=True)
                for use_graph in (False, True, True):
                    w.clear()
                    b.run(use_graph)
                    torch.cuda.synchronize()
                    assert BB.same(ref, w.snapshot()), (block, iw, kb, use_graph)
                    H.hf_run_solo(w.tasks[0], 512)  # eager work between replays
                b.close()
                ran += 1
    assert ran >= 14


def test_batch_schedule_search_gives_a_valid_schedule():
    kinds, logs, groups = BB.draw(50, seed=16, kmin=10, kmax=14)
    w = BB.Workload(kinds, logs, seed=16)
    ref = solo_reference(w)
    sched, ms, nprof = H.hf_batch_tune_sched(w.tasks, groups, reps=2)
    assert ms > 0 and nprof >= 30 and sched.block in (256, 512, 1024)
    b = H.Batch(w.tasks, groups, schedule=sched)
    for use_graph in (False, True):
        w.clear()
        b.run(use_graph)
        torch.cuda.synchronize()
        assert BB.same(ref, w.snapshot()), (sched.as_dict(), use_graph)
    b.close()


def test_batch_tune_gives_a_valid_schedule():
    kinds, logs, groups = BB.draw(50, seed=14, kmin=10, kmax=14)
    w = BB.Workload(kinds, logs, seed=14)
    ref = solo_reference(w)
    waves, block, ms = H.hf_batch_tune(w.tasks, groups, reps=3)
    assert block in (256, 512, 1024) and ms > 0
    b = H.Batch(w.tasks, groups, waves, block)
    w.clear()
    b.run(True)
    torch.cuda.synchronize()
    assert BB.same(ref, w.snapshot())
    b.close()


def test_full_batch_1000_instances():
    """1000 instances of 2^12..2^18 elements in groups of 2-4: every mode gives
    the back-to-back bits; sampled instances against the oracle."""
    kinds, logs, groups = BB.draw(1000, seed=3)
    w = BB.Workload(kinds, logs, seed=3)
    res, ref = BB.run_modes(w, groups, reps=2)
    print({k: v for k, v in res.items()}, flush=True)
    assert res["streams4_equal"] and res["graph_solo_equal"]
    assert res["batch_equal"] and res["batch_graph_equal"]
    for i in np.random.default_rng(0).choice(1000, 25, replace=False):
        check_instance(kinds[i], w.ins[i], ref[i])


def test_batch_with_hash_kinds():
    """Batches holding hash instances run the hash-capable kernel variant: the
    same bits as the solo launches, eager and from the graph."""
    kinds, logs, groups = BB.draw(48, seed=15, kmin=10, kmax=14, kinds=tuple(range(len(H.KIND_NAMES))))
    assert any(k >= H.HF_SHA256D for k in kinds)
    w = BB.Workload(kinds, logs, seed=15)
    ref = solo_reference(w)
    for k, x, o, m in zip(kinds, w.ins, ref, w.meta):
        check_instance(k, x, o, m)
    scheds = [(256, None), (1024, None), (512, H.hf_batch_schedule(512, 2, 64, 0)),
              (256, H.hf_batch_schedule(256, 1, 256, 0))]
    for block, sc in scheds:
        b = H.Batch(w.tasks, groups, None, block, schedule=sc)
        for graph in (False, True, True):
            w.clear()
            b.run(graph)
            torch.cuda.synchronize()
            assert BB.same(ref, w.snapshot()), (block, sc and sc.as_dict(), graph)
        b.close()
