"""GPU-resident velocity Verlet vs the oracle's integrator; energy
conservation; skin/rebuild policy vs rebuilding every step."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2405_01491_amd as nnp
from paper_2405_01491_amd import md as nmd
from tests.gpu_helpers import dev, to_dev

pytestmark = pytest.mark.gpu


def test_first_steps_track_oracle_trajectory(spec_bias):
    w = synthetic.workload(1)
    model = nnp.Model(spec_bias, "fp32")
    masses = synthetic.MASSES[w.species]
    v0 = nmd.maxwell_boltzmann(masses, 300.0, seed=5)
    pos, sp, _ = to_dev(w)
    sim = nmd.VelocityVerlet(model, pos.clone(), torch.from_numpy(v0).to(dev()), sp, masses, None, dt=0.5)
    for _ in range(10):
        sim.step()
    nl = oracle.neighbor_list(w.pos, None, None, 9.0)
    xr, vr, en = oracle.velocity_verlet(w.pos, v0, masses,
                                        lambda x: oracle.energy_forces_f64(x, w.species, None, spec_bias, nl),
                                        0.5, 10)
    x = sim.pos.cpu().numpy()
    v = sim.vel.cpu().numpy()
    print("10 steps: max |dx| %.3g A, max |dv| %.3g A/fs" % (np.abs(x - xr).max(), np.abs(v - vr).max()))
    assert np.abs(x - xr).max() < 1e-4
    assert np.abs(v - vr).max() < 1e-5
    assert abs(float(sim.e_mol[0]) - en[-1][0]) < 1e-4 * max(1.0, abs(en[-1][0]))


def test_nve_energy_conservation(spec):
    w = synthetic.geometry.small_water_box(64)
    model = nnp.Model(spec, "fp32")
    masses = synthetic.MASSES[w.species]
    pos, sp, _ = to_dev(w)
    v0 = torch.from_numpy(nmd.maxwell_boltzmann(masses, 300.0, seed=6)).to(dev())
    sim = nmd.VelocityVerlet(model, pos, v0, sp, masses, w.box, dt=0.25)
    E0 = sim.total_energy()
    Es = []
    for k in range(200):
        sim.step()
        if k % 20 == 19:
            Es.append(sim.total_energy())
    drift = max(abs(e - E0) for e in Es)
    ke = sim.kinetic_energy()
    print("NVE 200 steps: E0 %.6f drift %.3g eV (KE %.3g eV)" % (E0, drift, ke))
    assert drift < 0.02 * max(ke, 1.0)


def test_skin_policy_matches_rebuild_every_step(spec):
    w = synthetic.geometry.small_water_box(80)
    masses = synthetic.MASSES[w.species]
    v0 = nmd.maxwell_boltzmann(masses, 300.0, seed=7)
    res = []
    for skin, every in [(0.0, 1), (0.5, 20)]:
        model = nnp.Model(spec, "fp32")
        pos, sp, _ = to_dev(w)
        sim = nmd.VelocityVerlet(model, pos, torch.from_numpy(v0).to(dev()), sp, masses, w.box, dt=0.5,
                                 skin=skin, rebuild_every=every)
        for _ in range(40):
            sim.step()
        res.append((sim.pos.cpu().numpy(), float(sim.e_mol[0]), sim.rebuilds))
    # positions are wrapped at rebuilds: compare through the minimum image
    d = res[0][0] - res[1][0]
    d -= w.box * np.round(d / w.box)
    print("skin vs every-step after 40 steps: max |dx| %.3g A, rebuilds %d vs %d" % (np.abs(d).max(), res[0][2],
                                                                                    res[1][2]))
    assert np.abs(d).max() < 1e-4
    assert abs(res[0][1] - res[1][1]) < 1e-4 * max(1.0, abs(res[0][1]))
    assert res[1][2] < res[0][2]


def test_stage_profiling_counts(spec):
    w = synthetic.workload(1)
    model = nnp.Model(spec, "fp32")
    pos, sp, _ = to_dev(w)
    nmd.profile_enable(model, True)
    nl = nnp.nnp_neighbors(model, pos, None, 1, None, 5.1)
    for _ in range(3):
        nnp.nnp_energy_forces(model, pos, sp, None, 1, None, nl)
    st = nmd.profile_read(model)
    assert st["neighbors"][1] == 1 and st["aev"][1] == 3 and st["mlp"][1] == 3 and st["forces"][1] == 3
    assert all(v[0] >= 0 for v in st.values())
