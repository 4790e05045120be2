"""Neighbour list on the GPU vs the oracle: the pair set (i, j, image shift)
must be identical bit for bit; rows sorted; reverse index consistent; the
capacity / box / non-finite / mol error protocol."""
import types

import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2405_01491_amd as nnp
from paper_2405_01491_amd import _lib
from tests.gpu_helpers import dev, pairset, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model(spec):
    return nnp.Model(spec, "fp32")


def _check_list(nl, w, r_list):
    i, j, n = nl.pairs()
    ref = oracle.neighbor_list(w.pos, w.mol if w.n_mol > 1 else None, w.box, r_list)
    assert nl.n_pairs == len(ref[0]), (w.name, nl.n_pairs, len(ref[0]))
    assert pairset(i, j, n) == pairset(*ref), w.name
    # rows sorted by j, and identical order to the oracle's
    assert np.array_equal(i, ref[0]) and np.array_equal(j, ref[1]) and np.array_equal(n, ref[2])
    rev = nl.rev[:nl.n_pairs].cpu().numpy()
    assert np.array_equal(rev[rev], np.arange(nl.n_pairs))
    assert np.array_equal(j[rev], i) and np.array_equal(n[rev], -n)


@pytest.mark.parametrize("case", [c for c in synthetic.adversarial_cases() if c.name != "thin_box"],
                         ids=lambda c: c.name)
def test_adversarial_pair_sets(model, case):
    pos, sp, mol = to_dev(case)
    nl = nnp.nnp_neighbors(model, pos, mol, case.n_mol, case.box, 5.1)
    torch.cuda.synchronize()
    _check_list(nl, case, 5.1)


def test_thin_box_two_cells(model):
    case = [c for c in synthetic.adversarial_cases() if c.name == "thin_box"][0]
    pos, sp, mol = to_dev(case)
    nl = nnp.nnp_neighbors(model, pos, mol, 1, case.box, 5.1)
    _check_list(nl, case, 5.1)
    with pytest.raises(nnp.NNPError) as e:
        nnp.nnp_neighbors(model, pos, mol, 1, case.box, 5.6)
    assert e.value.status == _lib.NNP_E_BOX


@pytest.mark.parametrize("name,r_list", [("cluster", 5.1), ("cluster", 5.6), ("small_box", 5.6),
                                         ("water2", 5.1), ("water2", 5.6), ("serving", 5.1)])
def test_workload_pair_sets(model, name, r_list):
    w = {"cluster": lambda: synthetic.workload(1),
         "small_box": lambda: synthetic.geometry.small_water_box(64),
         "water2": lambda: synthetic.workload(2),
         "serving": lambda: synthetic.workload(4, n_mol=40)}[name]()
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(model, pos, mol, w.n_mol, w.box, r_list)
    _check_list(nl, w, r_list)


def test_dense_stencil_reads_candidates_from_global(model):
    """Periodic rows are built per cell from the stencil's atoms staged in
    LDS; a stencil holding more atoms than that stage (here the whole box:
    2,100 random atoms in a 19.9 A box, three cells of 1.3 r_list per side,
    about 150 neighbours per row) is searched from global memory row by
    row.  The list is exact either way."""
    rng = np.random.default_rng(31)
    L, n = 19.9, 2100
    w = types.SimpleNamespace(name="dense_box", pos=(rng.random((n, 3)) * L).astype(np.float32),
                              species=np.zeros(n, np.int32), mol=np.zeros(n, np.int32), n_mol=1,
                              box=np.array([L, L, L], np.float32), n_atoms=n)
    pos, sp, _ = to_dev(w)
    nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, 5.1)
    torch.cuda.synchronize()
    _check_list(nl, w, 5.1)
    assert np.diff(nl.row_ptr.cpu().numpy()).max() < 256


@pytest.mark.parametrize("cfg,r_list", [(3, 5.1), (5, 5.6)])
def test_large_pair_sets_sampled_rows(model, cfg, r_list):
    w = synthetic.workload(cfg)
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, r_list)
    rp = nl.row_ptr.cpu().numpy()
    col = nl.col[:nl.n_pairs].cpu().numpy()
    sh = nl.shift[:nl.n_pairs].cpu().numpy()
    rng = np.random.default_rng(cfg)
    rows = np.sort(rng.choice(w.n_atoms, size=300, replace=False))
    ri, rj, rn = oracle.neighbor_rows(w.pos, None, w.box, r_list, rows)
    for r in rows:
        sel = ri == r
        assert np.array_equal(col[rp[r]:rp[r + 1]], rj[sel]), r
        assert np.array_equal(sh[rp[r]:rp[r + 1]], rn[sel]), r
    # global properties at full size: symmetric list, sorted rows
    rev = nl.rev[:nl.n_pairs].cpu().numpy()
    assert np.array_equal(rev[rev], np.arange(nl.n_pairs))
    i = np.repeat(np.arange(w.n_atoms), np.diff(rp))
    assert np.array_equal(col[rev], i)
    key = i.astype(np.int64) * w.n_atoms + col
    assert np.all(np.diff(key) > 0)


def test_capacity_regrow(model):
    w = synthetic.workload(2)
    pos, sp, mol = to_dev(w)
    nl = nnp.NeighborList(w.n_atoms, 1000, dev())
    nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, 5.1, nl=nl)
    assert nl.regrows >= 1 and nl.capacity >= nl.n_pairs
    _check_list(nl, w, 5.1)


def test_nonfinite_and_bad_mol(model):
    w = synthetic.workload(1)
    pos, sp, _ = to_dev(w)
    bad = pos.clone()
    bad[5, 1] = float("nan")
    with pytest.raises(nnp.NNPError) as e:
        nnp.nnp_neighbors(model, bad, None, 1, None, 5.1)
    assert e.value.status == _lib.NNP_E_NONFINITE
    box = np.array([20.0, 20.0, 20.0], np.float32)
    with pytest.raises(nnp.NNPError) as e:
        nnp.nnp_neighbors(model, bad, None, 1, box, 5.1)
    assert e.value.status == _lib.NNP_E_NONFINITE
    two = torch.zeros(w.n_atoms, dtype=torch.int32, device=dev())
    two[w.n_atoms // 2:] = 1            # two structures: the ranges kernel also checks the coordinates
    with pytest.raises(nnp.NNPError) as e:
        nnp.nnp_neighbors(model, bad, two, 2, None, 5.1)
    assert e.value.status == _lib.NNP_E_NONFINITE
    mol = torch.zeros(w.n_atoms, dtype=torch.int32, device=dev())
    mol[10] = 1                         # 0..0 1 0..0: not non-decreasing
    with pytest.raises(nnp.NNPError) as e:
        nnp.nnp_neighbors(model, pos, mol, 2, None, 5.1)
    assert e.value.status == _lib.NNP_E_ARG
    # the flags were cleared: a good call succeeds afterwards
    nl = nnp.nnp_neighbors(model, pos, None, 1, None, 5.1)
    _check_list(nl, w, 5.1)


def test_empty_system(model):
    pos = torch.zeros((0, 3), dtype=torch.float32, device=dev())
    nl = nnp.nnp_neighbors(model, pos, None, 1, np.array([12.0, 12, 12], np.float32), 5.1)
    assert nl.n_pairs == 0
