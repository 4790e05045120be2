"""The allocation-free entry point (nnp_energy_forces_static) against
nnp_energy_forces, through the C ABI.

Both run the same kernels on the same inputs; only the scratch differs (the
library's fixed device array instead of the caller's workspace), so every
output must be identical bit for bit.  Two calls in a row, the second on a
smaller input, check that nothing in the shared scratch has to start at zero
(the second call reuses what the first left there)."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic
import paper_2405_01491_amd as nnp
from paper_2405_01491_amd import _lib
from tests.gpu_helpers import dev, to_dev

pytestmark = pytest.mark.gpu


def _plain(model, w, nl):
    pos, sp, mol = to_dev(w)
    e, ea, F = nnp.nnp_energy_forces(model, pos, sp, mol, w.n_mol, w.box, nl, e_atom=True)
    return e.cpu().numpy(), ea.cpu().numpy(), F.cpu().numpy()


def _static(model, w, nl, outs):
    """Direct ctypes call of the entry point into preallocated outputs."""
    L = _lib.lib()
    pos, sp, mol, e, ea, F = outs
    box = None if w.box is None else (ctypes.c_float * 3)(*np.asarray(w.box, np.float32).tolist())
    st = L.nnp_energy_forces_static(model.handle, w.n_atoms, ctypes.c_void_p(pos.data_ptr()),
                                    ctypes.c_void_p(sp.data_ptr()),
                                    None if mol is None else ctypes.c_void_p(mol.data_ptr()), w.n_mol, box,
                                    ctypes.byref(nl.struct()), ctypes.c_void_p(e.data_ptr()),
                                    ctypes.c_void_p(ea.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream))
    assert st == _lib.NNP_OK, _lib.STATUS_NAMES[st]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_static_equals_workspace_call_twice(spec_bias, precision):
    model = nnp.Model(spec_bias, precision)
    big = synthetic.geometry.small_water_box(1000)          # 3,000 atoms, periodic
    small = synthetic.workload(4, n_mol=12)                  # a batch of 12 open molecules, mol ids
    assert small.n_atoms < big.n_atoms
    d = dev()
    cases = []
    for w in (big, small):
        pos, sp, mol = to_dev(w)
        nl = nnp.nnp_neighbors(model, pos, mol, w.n_mol, w.box, 5.1)
        need = _lib.lib().nnp_workspace_bytes(model.handle, w.n_atoms, nl.capacity)
        assert need <= _lib.NNP_STATIC_SCRATCH_BYTES
        torch.cuda.synchronize()
        free_a = torch.cuda.mem_get_info(d)[0]
        want = _plain(model, w, nl)          # the workspace call: reference (and first launch of every kernel)
        torch.cuda.synchronize()
        print("%s %s: free device memory across the workspace call changed by %d bytes"
              % (precision, w.name, torch.cuda.mem_get_info(d)[0] - free_a))
        outs = (pos, sp, mol, torch.full((w.n_mol,), np.nan, dtype=torch.float64, device=d),
                torch.full((w.n_atoms,), np.nan, dtype=torch.float32, device=d),
                torch.full((w.n_atoms, 3), np.nan, dtype=torch.float32, device=d))
        cases.append((w, nl, want, outs))
    # two calls in a row on the shared scratch, the second on the smaller input
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(d)[0]
    for w, nl, _, outs in cases:
        _static(model, w, nl, outs)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(d)[0] == free0      # the calls took no device memory
    nnp.nnp_check(model)
    for w, nl, want, outs in cases:
        got = tuple(t.cpu().numpy() for t in outs[3:])
        for a, b, name in zip(got, want, ("e_mol", "e_atom", "forces")):
            assert np.all(np.isfinite(a)), name
            assert np.array_equal(a, b), (name, float(np.max(np.abs(a - b))))
        print("%s %s: %d atoms, %d structures, E = %.8f, identical to the workspace call"
              % (precision, w.name, w.n_atoms, w.n_mol, float(got[0].sum())))


def test_static_rejects_inputs_beyond_the_scratch(spec_bias):
    """A call whose intermediates exceed NNP_STATIC_SCRATCH_BYTES returns
    NNP_E_SCRATCH before anything is launched (the list here has no device
    arrays at all: nothing may touch them)."""
    L = _lib.lib()
    model = nnp.Model(spec_bias, "fp32")
    n = 20000
    nl = _lib.NList(row_ptr=None, col=None, shift=None, rev=None, capacity=80 * n, r_list=5.1, n_atoms=n,
                    n_pairs=0)
    assert L.nnp_workspace_bytes(model.handle, n, nl.capacity) > _lib.NNP_STATIC_SCRATCH_BYTES
    e = torch.empty(1, dtype=torch.float64, device=dev())
    st = L.nnp_energy_forces_static(model.handle, n, None, None, None, 1, None, ctypes.byref(nl),
                                    ctypes.c_void_p(e.data_ptr()), None, None,
                                    ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream))
    assert st == _lib.NNP_E_SCRATCH
    assert L.nnp_status_str(st) == b"input larger than the fixed scratch of the allocation-free call"
