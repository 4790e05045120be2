"""GPU-resident NVE molecular dynamics over the C ABI (Sec. 5.4, "Native MD
engine": velocity Verlet for NVE, state kept on the GPU, host only enqueues).

Per step:  kick + drift (nnp_md_kick_drift) -> neighbour rebuild when due
(wrap into the box, nnp_neighbors) -> energy and forces (nnp_energy_forces)
-> kick (nnp_md_kick).  With a skin (Sec. 5.5: a buffer and a rebuild every
few steps), the list is rebuilt every ``rebuild_every`` steps, and earlier if
the largest displacement since the last build exceeds ``trigger * skin / 2``
(two atoms that each moved less than half the skin cannot have closed the
gap).  That displacement is folded on the device after the drift and read
back before the step's forces are computed, so this driver waits once per
step when it has a skin; the native engine (``MDEngine``) decides on the
device and never waits.
"""
import ctypes

import numpy as np
import torch

from . import _lib, nnp_energy_forces, nnp_neighbors
from ._lib import check, lib

KB_EV = 8.617333262e-5       # eV / K
ACC_UNIT = 9.648533212e-3    # (eV / A / amu) -> A / fs^2


def maxwell_boltzmann(masses, temperature, seed):
    """Velocities (A/fs) at the given temperature, zero total momentum."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)
    sigma = np.sqrt(KB_EV * temperature / m * ACC_UNIT)
    v = rng.normal(size=(len(m), 3)) * sigma[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    return v.astype(np.float32)


def _s(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class VelocityVerlet:
    def __init__(self, model, pos, vel, species, masses, box=None, mol=None, n_mol=1, dt=0.5, skin=0.0,
                 rebuild_every=1, trigger=1.0):
        if skin > 0 and not (0 < trigger <= 1):
            raise ValueError("with a skin the displacement trigger must be in (0, 1]")
        if skin <= 0 and int(rebuild_every) != 1:
            raise ValueError("without a skin the list must be rebuilt every step")
        self.model = model
        self.dev = pos.device
        self.pos = pos.contiguous()
        self.vel = vel.contiguous()
        self.species = species
        self.mol = mol
        self.n_mol = n_mol
        self.box = None if box is None else np.asarray(box, dtype=np.float32)
        self._box_c = None if box is None else (ctypes.c_float * 3)(*self.box.tolist())
        self.inv_mass = (1.0 / torch.as_tensor(masses, dtype=torch.float32)).to(self.dev)
        self.dt = float(dt)
        self.skin = float(skin)
        self.r_list = float(model.spec.rc_r) + self.skin
        self.rebuild_every = max(1, int(rebuild_every))
        self.trigger2 = (trigger * 0.5 * self.skin) ** 2 if self.skin > 0 else None
        self.ref = torch.empty_like(self.pos)
        self.max_d2 = torch.zeros(1, dtype=torch.float32, device=self.dev)
        self._host_d2 = torch.zeros(1, dtype=torch.float32).pin_memory()
        self.out = {}
        self.nl = None
        self.steps = 0
        self.since_build = 0
        self.rebuilds = 0
        self.early_rebuilds = 0
        self._rebuild()
        self.e_mol, _, self.forces = nnp_energy_forces(model, self.pos, species, mol, n_mol, self.box, self.nl,
                                                       out=self.out)

    def _rebuild(self):
        L = lib()
        if self._box_c is not None:
            check(L.nnp_md_wrap(self.pos.shape[0], ctypes.c_void_p(self.pos.data_ptr()), self._box_c, _s(self.dev)),
                  "nnp_md_wrap")
        self.nl = nnp_neighbors(self.model, self.pos, self.mol, self.n_mol, self.box, self.r_list, nl=self.nl)
        self.ref.copy_(self.pos)
        self.max_d2.zero_()
        self.since_build = 0
        self.rebuilds += 1

    def step(self):
        L = lib()
        n = self.pos.shape[0]
        track = self.trigger2 is not None
        check(L.nnp_md_kick_drift(n, ctypes.c_void_p(self.pos.data_ptr()), ctypes.c_void_p(self.vel.data_ptr()),
                                  ctypes.c_void_p(self.forces.data_ptr()), ctypes.c_void_p(self.inv_mass.data_ptr()),
                                  ctypes.c_float(self.dt),
                                  ctypes.c_void_p(self.ref.data_ptr()) if track else None,
                                  ctypes.c_void_p(self.max_d2.data_ptr()) if track else None, _s(self.dev)),
              "nnp_md_kick_drift")
        self.since_build += 1
        due = self.since_build >= self.rebuild_every
        if not due and track:
            # this step's displacement, before its forces (NaN rebuilds, and
            # the rebuild then flags the coordinates)
            self._host_d2.copy_(self.max_d2, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record()
            ev.synchronize()
            d2 = float(self._host_d2[0])
            if not d2 <= self.trigger2:
                due = True
                self.early_rebuilds += 1
        if due:
            self._rebuild()
        self.e_mol, _, self.forces = nnp_energy_forces(self.model, self.pos, self.species, self.mol, self.n_mol,
                                                       self.box, self.nl, out=self.out)
        check(L.nnp_md_kick(n, ctypes.c_void_p(self.vel.data_ptr()), ctypes.c_void_p(self.forces.data_ptr()),
                            ctypes.c_void_p(self.inv_mass.data_ptr()), ctypes.c_float(self.dt), _s(self.dev)),
              "nnp_md_kick")
        self.steps += 1

    def kinetic_energy(self):
        m = 1.0 / self.inv_mass.double()
        return float(0.5 * (m[:, None] * self.vel.double() ** 2).sum() / ACC_UNIT)

    def total_energy(self):
        return float(self.e_mol.sum()) + self.kinetic_energy()


def profile_enable(model, enable=True, stages=None):
    """Time every stage (or only the named ones) of later calls."""
    if stages is None:
        check(lib().nnp_profile_enable(model.handle, 1 if enable else 0), "nnp_profile_enable")
    else:
        mask = sum(1 << _lib.STAGES.index(s) for s in stages) if enable else 0
        check(lib().nnp_profile_enable_mask(model.handle, mask), "nnp_profile_enable_mask")


def profile_read(model):
    ms = (ctypes.c_double * len(_lib.STAGES))()
    cnt = (ctypes.c_int64 * len(_lib.STAGES))()
    check(lib().nnp_profile_read(model.handle, ms, cnt), "nnp_profile_read")
    return {name: (ms[k], cnt[k]) for k, name in enumerate(_lib.STAGES)}


class MDEngine:
    """The native engine (nnp_md_*): NVE velocity Verlet or BAOAB Langevin
    dynamics with the whole step on the GPU; ``run(k)`` enqueues k steps and
    synchronises once.  State lives in the engine; ``state()`` copies it out."""

    def __init__(self, model, pos, vel, species, masses, box=None, dt=0.5, integrator="nve", temperature=300.0,
                 friction=1.0, seed=0, skin=0.0, rebuild_every=1, trigger=1.0, log_every=0, log_capacity=0):
        L = lib()
        self.model = model
        self.dev = pos.device
        self.n = pos.shape[0]
        m = torch.as_tensor(np.asarray(masses, dtype=np.float32)).to(self.dev)
        p = _lib.MdParams()
        p.integrator = {"nve": 0, "langevin": 1}[integrator]
        p.dt, p.temperature, p.friction, p.seed = float(dt), float(temperature), float(friction), int(seed)
        p.skin, p.rebuild_every, p.trigger = float(skin), int(rebuild_every), float(trigger)
        p.log_every, p.log_capacity = int(log_every), int(log_capacity)
        self.params = p
        self.box = None if box is None else np.asarray(box, dtype=np.float32)
        bptr = None if box is None else (ctypes.c_float * 3)(*self.box.tolist())
        h = ctypes.c_void_p()
        pos = pos.contiguous()
        vel = vel.contiguous()
        species = species.contiguous()
        with torch.cuda.device(self.dev):
            check(L.nnp_md_create(model.handle, self.n, ctypes.c_void_p(pos.data_ptr()),
                                  ctypes.c_void_p(vel.data_ptr()), ctypes.c_void_p(species.data_ptr()),
                                  ctypes.c_void_p(m.data_ptr()), bptr, ctypes.byref(p), _s(self.dev),
                                  ctypes.byref(h)), "nnp_md_create")
        self.handle = h

    def run(self, n_steps):
        with torch.cuda.device(self.dev):
            check(lib().nnp_md_run(self.handle, int(n_steps), _s(self.dev)), "nnp_md_run")

    def state(self):
        """(pos, vel, forces, e_pot) as new device tensors."""
        pos = torch.empty((self.n, 3), dtype=torch.float32, device=self.dev)
        vel = torch.empty_like(pos)
        F = torch.empty_like(pos)
        e = torch.empty(1, dtype=torch.float64, device=self.dev)
        with torch.cuda.device(self.dev):
            check(lib().nnp_md_get(self.handle, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()),
                                   ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(e.data_ptr()), _s(self.dev)),
                  "nnp_md_get")
        return pos, vel, F, e

    def log(self):
        """Logged rows [k, 2]: (E_pot, E_kin) in eV."""
        cap = max(int(self.params.log_capacity), 1)
        buf = np.zeros((cap, 2), dtype=np.float64)
        rows = ctypes.c_int32(0)
        check(lib().nnp_md_log(self.handle, ctypes.c_void_p(buf.ctypes.data), cap, ctypes.byref(rows),
                               _s(self.dev)), "nnp_md_log")
        return buf[:rows.value].copy()

    def info(self):
        st = _lib.MdStats()
        check(lib().nnp_md_info(self.handle, ctypes.byref(st), _s(self.dev)), "nnp_md_info")
        return {k: getattr(st, k) for k, _ in _lib.MdStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().nnp_md_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
