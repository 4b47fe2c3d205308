"""GPU parity of batched uneven expressions (2048 dot / matvec tasks in one
persistent launch, forward and backward) against the oracle, evaluated task by
task, plus the plain per-task form, autotuning, graph replay and edge cases."""
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import check_vector, say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


class Case:
    def __init__(self, bt):
        self.bt = bt
        self.tb = bt.table()
        self.A, self.B, self.g = dev(bt.A), dev(bt.B), dev(bt.gout)
        self.ref_out = O.batch_forward(self.tb, bt.A, bt.B, bt.out_len)
        self.S_out = O.batch_forward(self.tb, np.abs(bt.A), np.abs(bt.B), bt.out_len)
        m = np.zeros(bt.out_len)
        for t in range(bt.ntasks):
            m[bt.out_off[t]: bt.out_off[t] + (bt.rows[t] if bt.kind[t] else 1)] = bt.cols[t]
        self.m_out = m
        self.ref_gA, self.ref_gB = O.batch_backward(self.tb, bt.A, bt.B, bt.gout)
        _, self.S_gB = O.batch_backward(self.tb, np.abs(bt.A), np.abs(bt.B), np.abs(bt.gout))
        mb = np.ones(bt.B.size)
        for t in range(bt.ntasks):
            if bt.kind[t]:
                mb[bt.b_off[t]: bt.b_off[t] + bt.cols[t]] = bt.rows[t]
        self.m_gB = mb
        # elements that belong to some task (the pools may hold padding between
        # operands, which no call may write)
        self.in_A = np.zeros(bt.A.size, dtype=bool)
        self.in_B = np.zeros(bt.B.size, dtype=bool)
        for t in range(bt.ntasks):
            self.in_A[bt.a_off[t]: bt.a_off[t] + bt.rows[t] * bt.cols[t]] = True
            self.in_B[bt.b_off[t]: bt.b_off[t] + bt.cols[t]] = True

    def check(self, out, gA, gB, what):
        check_vector(host(out), self.ref_out, self.S_out, self.m_out, what=what + " out")
        # every gradient element of A (and of B for dots) is one binary32 product
        hA, hB = host(gA), host(gB)
        assert np.array_equal(hA[self.in_A], self.ref_gA[self.in_A].astype(np.float32)), what + " gA"
        check_vector(hB[self.in_B], self.ref_gB[self.in_B], self.S_gB[self.in_B], self.m_gB[self.in_B],
                     what=what + " gB")
        # the padding between operands was filled with NaN and must stay so
        assert np.isnan(hA[~self.in_A]).all() and np.isnan(hB[~self.in_B]).all(), what + " padding written"


@pytest.fixture(scope="module")
def config_case():
    say("batch config case: 2048 tasks, sizes log-uniform 1e2..1e6")
    return Case(W.batched_tasks(2048, seed=0))


def run(case, batch, plain=False):
    bt = case.bt
    out = torch.full((bt.out_len,), float("nan"), device=DEV)
    gA = torch.full((bt.A.size,), float("nan"), device=DEV)
    gB = torch.full((bt.B.size,), float("nan"), device=DEV)
    batch.forward(case.A, case.B, out, plain=plain)
    batch.backward(case.A, case.B, case.g, gA, gB, plain=plain)
    return out, gA, gB


def test_batch_config_persistent(config_case):
    say("batch persistent")
    b = api.Batch(config_case.tb)
    config_case.check(*run(config_case, b), "persistent")


def test_batch_config_unpadded_pools():
    """The full 2048-task configuration with operands packed back to back (odd
    offsets, so most tasks start off any 16-byte boundary): forward and
    backward in the persistent launch against the oracle."""
    say("batch config unpadded pools")
    case = Case(W.batched_tasks(2048, seed=1, pad=1))
    assert np.any(case.bt.a_off % 4 != 0) and np.any(case.bt.b_off % 2 == 1)
    b = api.Batch(case.tb)
    case.check(*run(case, b), "unpadded")


def test_batch_config_plain(config_case):
    say("batch plain")
    b = api.Batch(config_case.tb)
    config_case.check(*run(config_case, b, plain=True), "plain")


@pytest.mark.parametrize("cfg", [(4096, 2), (8192, 16), (65536, 4), (1 << 20, 1)])
def test_batch_configs_agree(config_case, cfg):
    say("batch cfg", cfg)
    b = api.Batch(config_case.tb, cfg)
    assert b.config == cfg
    config_case.check(*run(config_case, b), f"cfg {cfg}")


def test_batch_deterministic_and_permutation_invariant(config_case):
    say("batch permutation")
    b = api.Batch(config_case.tb)
    o1, a1, g1 = (host(t) for t in run(config_case, b))
    o2, a2, g2 = (host(t) for t in run(config_case, b))
    assert o1.tobytes() == o2.tobytes() and g1.tobytes() == g2.tobytes()
    perm = np.random.default_rng(0).permutation(config_case.bt.ntasks)
    bp = api.Batch(config_case.tb[perm])
    o3, a3, g3 = (host(t) for t in run(config_case, bp))
    assert o1.tobytes() == o3.tobytes() and a1.tobytes() == a3.tobytes() and g1.tobytes() == g3.tobytes()


def test_batch_autotune_and_cache(config_case, tmp_path):
    say("batch autotune")
    b = api.Batch(config_case.tb)
    bt = config_case.bt
    out = torch.empty(bt.out_len, device=DEV)
    gA = torch.empty(bt.A.size, device=DEV)
    gB = torch.empty(bt.B.size, device=DEV)
    cache = str(tmp_path / "tune.jsonl")
    chosen = b.autotune(config_case.A, config_case.B, out, config_case.g, gA, gB, cache_path=cache)
    assert os.path.exists(cache) and b.config == chosen
    config_case.check(*run(config_case, b), "autotuned")
    b2 = api.Batch(config_case.tb)
    assert b2.autotune(config_case.A, config_case.B, out, config_case.g, gA, gB, cache_path=cache) == chosen
    assert len(open(cache).read().strip().splitlines()) == 1  # served from the cache


def test_batch_graph_replay(config_case):
    say("batch graph")
    b = api.Batch(config_case.tb)
    bt = config_case.bt
    # the pools' padding belongs to no task and is never written: start every
    # run from the same NaN fill so that the byte comparison covers it too
    out = torch.full((bt.out_len,), float("nan"), device=DEV)
    gA = torch.full((bt.A.size,), float("nan"), device=DEV)
    gB = torch.full((bt.B.size,), float("nan"), device=DEV)
    b.forward(config_case.A, config_case.B, out)
    b.backward(config_case.A, config_case.B, config_case.g, gA, gB)
    ref = [host(out).copy(), host(gA).copy(), host(gB).copy()]
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        abi.mx_graph_begin(side)
        b.forward(config_case.A, config_case.B, out, stream=side)
        b.backward(config_case.A, config_case.B, config_case.g, gA, gB, stream=side)
        graph = abi.mx_graph_end(side)
    for rep in range(3):
        out.fill_(float("nan"))
        gA.fill_(float("nan"))
        gB.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(side)
        side.synchronize()
        for a, r in zip((host(out), host(gA), host(gB)), ref):
            assert a.tobytes() == r.tobytes(), rep
        b.forward(config_case.A, config_case.B, out)  # eager work between replays
        torch.cuda.synchronize()
    abi.mx_graph_destroy(graph)


def test_batch_edge_cases():
    say("batch edges")
    # empty dot, empty matvec (0 rows), one-element dot, a long dot spanning many tiles
    table = np.array([[0, 1, 0, 0, 0, 0],
                      [1, 0, 7, 0, 0, 1],
                      [0, 1, 1, 0, 7, 1],
                      [0, 1, 300001, 1, 8, 2],
                      [1, 5, 3, 300002, 300009, 3]], dtype=np.int64)
    rng = np.random.default_rng(0)
    A = rng.uniform(-1, 1, 300017).astype(np.float32)
    Bv = rng.uniform(-1, 1, 300012).astype(np.float32)
    g = rng.uniform(-1, 1, 8).astype(np.float32)
    b = api.Batch(table, (4096, 4))
    out = torch.zeros(8, device=DEV)
    gA = torch.zeros(A.size, device=DEV)
    gB = torch.zeros(Bv.size, device=DEV)
    b.forward(dev(A), dev(Bv), out)
    b.backward(dev(A), dev(Bv), dev(g), gA, gB)
    ref = O.batch_forward(table, A, Bv, 8)
    S = O.batch_forward(table, np.abs(A), np.abs(Bv), 8)
    check_vector(host(out), ref, S, np.array([1, 1, 300001, 3, 3, 3, 3, 3]), what="edge out")
    rA, rB = O.batch_backward(table, A, Bv, g)
    assert np.array_equal(host(gA), rA.astype(np.float32))
    SB = O.batch_backward(table, np.abs(A), np.abs(Bv), np.abs(g))[1]
    check_vector(host(gB), rB, SB, np.ones(Bv.size) * 5, what="edge gB")
    with pytest.raises(abi.MxError):
        api.Batch(np.array([[0, 2, 5, 0, 0, 0]]))  # a dot must have rows = 1
    empty = api.Batch(np.zeros((0, 6), dtype=np.int64))
    empty.forward(dev(A), dev(Bv), out)
