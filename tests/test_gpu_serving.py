"""Continuous-batching server: each result is the same alone and in the mix,
no ticket is lost or duplicated, out-of-order polling, memory/slot admission,
invalid requests, and batching of requests that arrive while others run."""
import time

import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2405_01491_amd as nnp
from paper_2405_01491_amd import _lib
from paper_2405_01491_amd.server import Server, nnp_poll, nnp_submit
from tests.gpu_helpers import F_MAX_ABS, dev

pytestmark = pytest.mark.gpu


def _wait(server, tickets, timeout=30.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = nnp_poll(server, t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not complete requests"
    return out


@pytest.fixture(scope="module")
def model(spec_bias):
    return nnp.Model(spec_bias, "fp32")


def _alone(model, p, s):
    pk = torch.from_numpy(p).to(dev())
    sk = torch.from_numpy(s).to(dev())
    nl = nnp.nnp_neighbors(model, pk, None, 1, None, model.spec.rc_r)
    e, _, f = nnp.nnp_energy_forces(model, pk, sk, None, 1, None, nl)
    return float(e[0]), f.cpu().numpy()


def test_results_same_alone_and_in_mix(model, spec_bias):
    rng = np.random.default_rng(101)
    mols = [synthetic.serving_molecule(rng) for _ in range(60)]
    srv = Server(model, max_inflight=2)
    tickets = [nnp_submit(srv, s, p) for p, s in mols]          # a burst: batched launches
    assert len(set(tickets)) == len(tickets) and tickets == sorted(tickets)
    res = _wait(srv, list(reversed(tickets)))                   # poll out of order
    st = srv.stats()
    print("burst of 60: %d launches, %d requests batched" % (st["launches"], st["batched_requests"]))
    assert st["completed"] == 60 and st["batched_requests"] == 60
    assert st["launches"] < 60                                   # requests shared launches
    for (p, s), t in zip(mols, tickets):
        e_mix, f_mix = res[t]
        e_alone, f_alone = _alone(model, p, s)
        assert abs(e_mix - e_alone) <= 1e-12 * max(1.0, abs(e_alone))
        assert np.array_equal(f_mix, f_alone)
    # and against the oracle for a few of them
    for k in (0, 17, 59):
        p, s = mols[k]
        ref = oracle.energy_forces(p, s, None, 1, None, spec_bias)
        e, f = res[tickets[k]]
        assert abs(e - ref["E_mol"][0]) <= 1e-5 * max(1.0, abs(ref["E_mol"][0]))
        assert np.abs(f - ref["F"]).max() < F_MAX_ABS
    # a collected ticket cannot be polled again
    with pytest.raises(KeyError):
        nnp_poll(srv, tickets[0])
    srv.close()


def test_admission_by_memory_and_slots(model):
    rng = np.random.default_rng(5)
    mols = [synthetic.serving_molecule(rng, n=100) for _ in range(8)]
    # arena for ~3 molecules of 100 atoms (16 B per atom)
    srv = Server(model, arena_bytes=3 * 1600 + 100, max_slots=5, max_inflight=1)
    acc = []
    busy = 0
    for p, s in mols:
        t = nnp_submit(srv, s, p)
        if t is None:
            busy += 1
        else:
            acc.append(t)
    assert busy > 0 and len(acc) >= 3
    _wait(srv, acc)
    # memory and slots free up after completion: admitted again
    t = nnp_submit(srv, mols[-1][1], mols[-1][0])
    assert t is not None
    _wait(srv, [t])
    # slot limit: with the arena large enough, the 6th unpolled request is refused
    srv2 = Server(model, arena_bytes=1 << 20, max_slots=5, max_inflight=1)
    ts = [nnp_submit(srv2, s, p) for p, s in mols[:6]]
    assert ts[:5] == [x for x in ts[:5] if x is not None] and ts[5] is None
    _wait(srv2, ts[:5])
    srv.close()
    srv2.close()


def test_invalid_requests(model):
    srv = Server(model, max_inflight=1)
    p = np.zeros((3, 3), np.float32)
    with pytest.raises(nnp.NNPError):
        nnp_submit(srv, np.array([0, 1, 9], np.int32), p)
    with pytest.raises(nnp.NNPError):
        nnp_submit(srv, np.zeros(300, np.int32), np.zeros((300, 3), np.float32))
    p[1, 2] = np.nan
    with pytest.raises(nnp.NNPError) as e:
        nnp_submit(srv, np.array([0, 1, 3], np.int32), p)
    assert e.value.status == _lib.NNP_E_NONFINITE
    # single atom: energy is the output bias + self energy; zero force
    t = nnp_submit(srv, np.array([2], np.int32), np.zeros((1, 3), np.float32))
    e, f = _wait(srv, [t])[t]
    assert np.all(f == 0.0)
    srv.close()


def test_requests_arriving_while_running_join_later_launches(model):
    rng = np.random.default_rng(9)
    srv = Server(model, max_inflight=2)
    mols = [synthetic.serving_molecule(rng) for _ in range(200)]
    tickets = []
    for k, (p, s) in enumerate(mols):
        tickets.append(nnp_submit(srv, s, p))
        if k % 20 == 19:
            time.sleep(0.002)
    _wait(srv, tickets)
    st = srv.stats()
    print("stream of 200: %d launches" % st["launches"])
    assert st["completed"] == 200 and st["launches"] >= 2
    srv.close()
