"""MI355X (gfx950) AEV neural-network potential: energy and forces.

A thin Python layer over libnnp's C ABI (include/nnp.h).  PyTorch provides
device memory and streams; every step of the computation runs in the HIP
kernels of libnnp.  The functions carry the C names:

    nnp_neighbors(model, pos, ...)        -> NeighborList
    nnp_energy_forces(model, pos, ...)    -> (e_mol, e_atom, forces)
    nnp_aev(model, pos, species, ...)     -> aev rows
    nnp_mlp(model, species, aev)          -> (e_atom, daev)
    nnp_submit / nnp_poll                 (see server.py)

plus ``Model`` (weights on the device), ``NeighborList`` (caller-owned list
buffers with the regrow-on-capacity protocol of Sec. 2.1's padded lists),
``NNPEnergy`` (a torch.autograd.Function whose backward returns minus the
forces) and ``md.VelocityVerlet`` (GPU-resident NVE dynamics).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import NNPError, NNP_FP32, NNP_BF16_MLP, NNP_E_CAPACITY, check, lib

__all__ = [
    "Model", "NeighborList", "nnp_neighbors", "nnp_energy_forces", "nnp_aev", "nnp_mlp",
    "NNPEnergy", "energy", "NNPError", "NNP_FP32", "NNP_BF16_MLP", "nnp_check",
]

_PRECISIONS = {"fp32": NNP_FP32, "bf16": NNP_BF16_MLP, NNP_FP32: NNP_FP32, NNP_BF16_MLP: NNP_BF16_MLP}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _box_arg(box):
    if box is None:
        return None, None
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float32).reshape(3))
    return b, b.ctypes.data_as(ctypes.c_void_p)


class Model:
    """Device-resident model.  ``spec`` provides the AEV hyper-parameters
    (n_species, rc_r, eta_r, shf_r, rc_a, eta_a, zeta, shf_a, shf_z,
    radial_prefactor, cos_scale), the layer ``widths``, ``celu_alpha``, the
    per-species ``weights`` [species][layer] = (W [out,in], b [out]) and
    optional ``self_energy``."""

    def __init__(self, spec, precision="fp32", device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.spec = spec
        L = lib()
        keep = []

        def fp(a):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
            keep.append(a)
            return a.ctypes.data_as(_lib.c_float_p)

        ap = _lib.AevParams(
            n_species=spec.n_species, rc_r=spec.rc_r, eta_r=spec.eta_r, n_shf_r=len(spec.shf_r),
            shf_r=fp(spec.shf_r), rc_a=spec.rc_a, eta_a=spec.eta_a, zeta=spec.zeta,
            n_shf_a=len(spec.shf_a), n_shf_z=len(spec.shf_z), shf_a=fp(spec.shf_a), shf_z=fp(spec.shf_z),
            radial_prefactor=spec.radial_prefactor, cos_scale=spec.cos_scale)
        n_layers = len(spec.widths) - 1
        widths = np.ascontiguousarray(np.asarray(spec.widths, dtype=np.int32))
        se = None
        if getattr(spec, "self_energy", None) is not None:
            se_arr = np.ascontiguousarray(np.asarray(spec.self_energy, dtype=np.float64))
            keep.append(se_arr)
            se = se_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        # an ensemble spec lists every network's weights; a plain spec has one network
        nets = getattr(spec, "ensemble", None) or [spec.weights]
        mps = (_lib.MlpParams * len(nets))()
        for k, weights in enumerate(nets):
            Ws = (_lib.c_float_p * (spec.n_species * n_layers))()
            bs = (_lib.c_float_p * (spec.n_species * n_layers))()
            keep.extend([Ws, bs])
            for s in range(spec.n_species):
                for l in range(n_layers):
                    W, b = weights[s][l]
                    Ws[s * n_layers + l] = fp(W)
                    bs[s * n_layers + l] = fp(b)
            mps[k] = _lib.MlpParams(n_layers=n_layers, widths=widths.ctypes.data_as(_lib.c_int32_p), W=Ws, b=bs,
                                    celu_alpha=spec.celu_alpha, self_energy=se)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.nnp_model_create_ensemble(ctypes.byref(ap), mps, len(nets), _PRECISIONS[precision],
                                              ctypes.byref(handle)), "nnp_model_create_ensemble")
        self.handle = handle
        self.n_nets = int(L.nnp_model_nets(handle))
        self.precision = precision
        self.aev_dim = L.nnp_aev_dim(handle)
        self.aev_stride = (self.aev_dim + 63) // 64 * 64
        self._ws = None

    def set_precision(self, precision):
        check(lib().nnp_model_set_precision(self.handle, _PRECISIONS[precision]), "nnp_model_set_precision")
        self.precision = precision

    @property
    def fused_mlp(self):
        return bool(lib().nnp_model_fused_mlp(self.handle))

    def set_fused_mlp(self, allow):
        check(lib().nnp_model_set_fused_mlp(self.handle, 1 if allow else 0), "nnp_model_set_fused_mlp")

    def workspace(self, nbytes):
        """A device byte buffer of at least nbytes, reused across calls on the
        same stream (kernels on one stream run in order)."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def close(self):
        if getattr(self, "handle", None):
            lib().nnp_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NeighborList:
    """Caller-owned CSR neighbour list on the device (row_ptr, col, shift,
    rev) with a capacity that grows by a multiplicative factor when a build
    reports NNP_E_CAPACITY (the running-maximum padding of Sec. 2.1)."""

    def __init__(self, n_atoms, capacity, device, growth=1.25):
        self.device = device
        self.growth = growth
        self.n_atoms = n_atoms
        self.row_ptr = torch.zeros(n_atoms + 1, dtype=torch.int32, device=device)
        self._alloc(capacity)
        self.c = _lib.NList()
        self.rebuilds = 0
        self.regrows = 0

    def _alloc(self, capacity):
        capacity = max(int(capacity), 1)
        self.capacity = capacity
        self.col = torch.empty(capacity, dtype=torch.int32, device=self.device)
        self.shift = torch.empty((capacity, 3), dtype=torch.int8, device=self.device)
        self.rev = torch.empty(capacity, dtype=torch.int32, device=self.device)

    def struct(self):
        c = self.c
        c.row_ptr = self.row_ptr.data_ptr()
        c.col = self.col.data_ptr()
        c.shift = self.shift.data_ptr()
        c.rev = self.rev.data_ptr()
        c.capacity = self.capacity
        return c

    @property
    def n_pairs(self):
        return int(self.c.n_pairs)

    @property
    def r_list(self):
        return float(self.c.r_list)

    def pairs(self):
        """(i, j, shift) as CPU numpy arrays, rows in order."""
        n = self.n_pairs
        rp = self.row_ptr.cpu().numpy().astype(np.int64)
        i = np.repeat(np.arange(self.n_atoms), np.diff(rp))
        return i, self.col[:n].cpu().numpy().astype(np.int64), self.shift[:n].cpu().numpy().astype(np.int64)


def nnp_neighbors(model, pos, mol=None, n_mol=1, box=None, r_list=None, nl=None, capacity=None):
    """Build (or rebuild into ``nl``) the neighbour list.  One host
    synchronisation; regrows the capacity and retries on NNP_E_CAPACITY."""
    L = lib()
    n = pos.shape[0]
    if r_list is None:
        r_list = model.spec.rc_r
    if nl is None or nl.n_atoms != n:
        nl = NeighborList(n, capacity if capacity else max(64 * n, 64), pos.device)
    _b, bptr = _box_arg(box)
    nmol = int(n_mol) if mol is not None else 1
    need = L.nnp_neighbors_workspace_bytes(n, nmol, bptr, ctypes.c_float(r_list))
    if need == 0 and box is not None:
        raise NNPError(_lib.NNP_E_BOX, "nnp_neighbors_workspace_bytes")
    ws = model.workspace(need)
    npairs = ctypes.c_int64(0)
    with torch.cuda.device(pos.device):
        for _attempt in range(8):
            st = L.nnp_neighbors(model.handle, n, _ptr(pos), _ptr(mol), nmol, bptr, ctypes.c_float(r_list),
                                 ctypes.byref(nl.struct()), ctypes.byref(npairs), _ptr(ws), ws.numel(),
                                 _stream(pos.device))
            if st == NNP_E_CAPACITY:
                nl._alloc(int(npairs.value * nl.growth) + 64)
                nl.regrows += 1
                continue
            check(st, "nnp_neighbors")
            nl.rebuilds += 1
            return nl
    raise NNPError(NNP_E_CAPACITY, "nnp_neighbors")


def nnp_energy_forces(model, pos, species, mol=None, n_mol=1, box=None, nl=None, forces=True, e_atom=False,
                      out=None, virial=False, atom_virial=False):
    """Energies (float64 [n_mol]), optional atomic energies (float32 [N]) and
    forces (float32 [N,3]); asynchronous on the current stream.  With
    ``virial`` (or ``atom_virial``) the virial W = -sum_edges v_ij (outer)
    dE_i/dv_ij per structure (float64 [n_mol,3,3]) and, if asked, per atom
    (float32 [N,3,3]) are stored in ``out["virial"]`` / ``out["atom_virial"]``."""
    L = lib()
    n = pos.shape[0]
    if nl is None:
        nl = nnp_neighbors(model, pos, mol, n_mol, box)
    dev = pos.device
    if out is None:
        out = {}
    e_mol_t = out.get("e_mol")
    if e_mol_t is None or e_mol_t.numel() != n_mol:
        e_mol_t = torch.empty(n_mol, dtype=torch.float64, device=dev)
    e_at = None
    if e_atom:
        e_at = out.get("e_atom")
        if e_at is None or e_at.numel() != n:
            e_at = torch.empty(n, dtype=torch.float32, device=dev)
    F = None
    if forces:
        F = out.get("forces")
        if F is None or F.shape[0] != n:
            F = torch.empty((n, 3), dtype=torch.float32, device=dev)
    _b, bptr = _box_arg(box)
    need = L.nnp_workspace_bytes(model.handle, n, nl.capacity)
    ws = model.workspace(need)
    if virial or atom_virial:
        if F is None:
            raise ValueError("the virial comes from the force adjoint: forces=True is required")
        W = out.get("virial")
        if W is None or W.shape[0] != n_mol:
            W = torch.empty((n_mol, 3, 3), dtype=torch.float64, device=dev)
        Wa = None
        if atom_virial:
            Wa = out.get("atom_virial")
            if Wa is None or Wa.shape[0] != n:
                Wa = torch.empty((n, 3, 3), dtype=torch.float32, device=dev)
        with torch.cuda.device(dev):
            check(L.nnp_energy_forces_virial(model.handle, n, _ptr(pos), _ptr(species), _ptr(mol), int(n_mol), bptr,
                                             ctypes.byref(nl.struct()), _ptr(e_mol_t), _ptr(e_at), _ptr(F), _ptr(W),
                                             _ptr(Wa), _ptr(ws), ws.numel(), _stream(dev)),
                  "nnp_energy_forces_virial")
        out.update(e_mol=e_mol_t, e_atom=e_at, forces=F, virial=W, atom_virial=Wa)
        return e_mol_t, e_at, F
    with torch.cuda.device(dev):
        check(L.nnp_energy_forces(model.handle, n, _ptr(pos), _ptr(species), _ptr(mol), int(n_mol), bptr,
                                  ctypes.byref(nl.struct()), _ptr(e_mol_t), _ptr(e_at), _ptr(F), _ptr(ws),
                                  ws.numel(), _stream(dev)), "nnp_energy_forces")
    out.update(e_mol=e_mol_t, e_atom=e_at, forces=F)
    return e_mol_t, e_at, F


def nnp_energy_forces_static(model, pos, species, mol=None, n_mol=1, box=None, nl=None, e_atom=None, forces=None,
                             e_mol=None):
    """nnp_energy_forces through the allocation-free entry point: the library
    works in its fixed device scratch (NNP_STATIC_SCRATCH_BYTES), and the
    caller passes every output buffer (e_mol float64 [n_mol], forces float32
    [N,3] or None, e_atom float32 [N] or None), so this wrapper allocates
    nothing when they are given.  Calls overlapping on one device race."""
    L = lib()
    n = pos.shape[0]
    dev = pos.device
    if e_mol is None:
        e_mol = torch.empty(n_mol, dtype=torch.float64, device=dev)
    _b, bptr = _box_arg(box)
    with torch.cuda.device(dev):
        check(L.nnp_energy_forces_static(model.handle, n, _ptr(pos), _ptr(species), _ptr(mol), int(n_mol), bptr,
                                         ctypes.byref(nl.struct()), _ptr(e_mol), _ptr(e_atom), _ptr(forces),
                                         _stream(dev)), "nnp_energy_forces_static")
    return e_mol, e_atom, forces


def nnp_energy_forces_ensemble(model, pos, species, mol=None, n_mol=1, box=None, nl=None, forces=True,
                               e_atom=False):
    """Ensemble-mean energies / forces plus every network's structure
    energies (float64 [n_nets, n_mol])."""
    L = lib()
    n = pos.shape[0]
    if nl is None:
        nl = nnp_neighbors(model, pos, mol, n_mol, box)
    dev = pos.device
    e_mol = torch.empty(n_mol, dtype=torch.float64, device=dev)
    e_net = torch.empty((model.n_nets, n_mol), dtype=torch.float64, device=dev)
    e_at = torch.empty(n, dtype=torch.float32, device=dev) if e_atom else None
    F = torch.empty((n, 3), dtype=torch.float32, device=dev) if forces else None
    _b, bptr = _box_arg(box)
    ws = model.workspace(L.nnp_workspace_bytes(model.handle, n, nl.capacity))
    with torch.cuda.device(dev):
        check(L.nnp_energy_forces_ensemble(model.handle, n, _ptr(pos), _ptr(species), _ptr(mol), int(n_mol), bptr,
                                           ctypes.byref(nl.struct()), _ptr(e_mol), _ptr(e_net), _ptr(e_at),
                                           _ptr(F), _ptr(ws), ws.numel(), _stream(dev)),
              "nnp_energy_forces_ensemble")
    return e_mol, e_net, e_at, F


def nnp_aev(model, pos, species, box=None, nl=None):
    """AEV rows [N, stride] (float32, atom order, zero padding columns)."""
    L = lib()
    n = pos.shape[0]
    if nl is None:
        nl = nnp_neighbors(model, pos, None, 1, box)
    A = torch.empty((n, model.aev_stride), dtype=torch.float32, device=pos.device)
    _b, bptr = _box_arg(box)
    with torch.cuda.device(pos.device):
        check(L.nnp_aev(model.handle, n, _ptr(pos), _ptr(species), bptr, ctypes.byref(nl.struct()), _ptr(A),
                        None, 0, _stream(pos.device)), "nnp_aev")
    return A


def nnp_mlp(model, species, aev, grad=True):
    """Species networks on given AEV rows [N, stride]: (e_atom [N], dE/dAEV)."""
    L = lib()
    n = species.shape[0]
    dev = species.device
    e = torch.empty(n, dtype=torch.float32, device=dev)
    g = torch.empty((n, model.aev_stride), dtype=torch.float32, device=dev) if grad else None
    need = L.nnp_workspace_bytes(model.handle, n, 0)
    ws = model.workspace(need)
    with torch.cuda.device(dev):
        check(L.nnp_mlp(model.handle, n, _ptr(species), _ptr(aev.contiguous()), _ptr(e), _ptr(g), _ptr(ws),
                        ws.numel(), _stream(dev)), "nnp_mlp")
    return e, g


def nnp_check(model, device=None):
    """Synchronise and raise if a device-side error flag is set."""
    flags = ctypes.c_uint32(0)
    check(lib().nnp_check(model.handle, _stream(device), ctypes.byref(flags)), "nnp_check")
    return flags.value


class NNPEnergy(torch.autograd.Function):
    """E_mol(pos) with dE/dpos = -forces.  Structures do not interact (atoms
    of different structures never share an edge), so the vector-Jacobian
    product is -F_a * g[mol_a]."""

    @staticmethod
    def forward(ctx, pos, species, mol, n_mol, box, model, nl):
        e_mol, _, F = nnp_energy_forces(model, pos.detach(), species, mol, n_mol, box, nl, forces=True)
        ctx.save_for_backward(F, mol)
        return e_mol

    @staticmethod
    def backward(ctx, g):
        F, mol = ctx.saved_tensors
        gm = g.to(torch.float32)
        ga = gm[mol.long()] if mol is not None else gm.expand(F.shape[0])
        return -F * ga[:, None], None, None, None, None, None, None


def energy(model, pos, species, mol=None, n_mol=1, box=None, nl=None):
    """Differentiable structure energies (see NNPEnergy)."""
    if nl is None:
        nl = nnp_neighbors(model, pos.detach(), mol, n_mol, box)
    return NNPEnergy.apply(pos, species, mol, n_mol, box, model, nl)
