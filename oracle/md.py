"""Oracle integrators of the native MD engine (Sec. 5.4, "Native MD engine":
velocity Verlet for NVE dynamics, BAOAB for Langevin dynamics; Sec. 5.5 runs
its benchmarks with a Langevin thermostat at 300 K).

Velocity Verlet:
    v(t + dt/2) = v(t) + dt/2 a(t)
    x(t + dt)   = x(t) + dt v(t + dt/2)
    v(t + dt)   = v(t + dt/2) + dt/2 a(t + dt),      a = F / m
BAOAB (Leimkuhler and Matthews), one step:
    B: v += dt/2 a;  A: x += dt/2 v;
    O: v = c1 v + sqrt(1 - c1^2) sqrt(kT / m) xi,  c1 = exp(-gamma dt);
    A: x += dt/2 v;  forces;  B: v += dt/2 a.
The Gaussian numbers xi of atom a at step s are taken from one block of the
counter-based generator Philox4x64-10 (numpy's implementation) with counter
(a + 1, s, 0, 0) and key (seed, 0): with the block's 64-bit words w_k,
u_k = ((w_k >> 40) + 1/2) 2^-24, and Box-Muller gives
xi = (rho0 cos 2 pi u1, rho0 sin 2 pi u1, rho2 cos 2 pi u3), rho_k = sqrt(-2 ln u_k).

Units: A, fs, amu, eV; 1 eV/(A amu) = 9.648533212e-3 A/fs^2.
"""
import numpy as np

ACC_UNIT = 9.648533212e-3      # (eV / A / amu) -> A / fs^2
KB_EV = 8.617333262e-5         # eV / K


def velocity_verlet(pos, vel, masses, force_fn, dt, n_steps):
    """Integrate n_steps in float64.  ``force_fn(x) -> (E_pot, F)``.
    Returns positions, velocities and (E_pot, E_kin) per step (step 0 first)."""
    x = np.asarray(pos, dtype=np.float64).copy()
    v = np.asarray(vel, dtype=np.float64).copy()
    m = np.asarray(masses, dtype=np.float64)[:, None]
    E, F = force_fn(x)
    energies = [(E, 0.5 * np.sum(m * v * v) / ACC_UNIT)]
    for _ in range(n_steps):
        v += 0.5 * dt * ACC_UNIT * F / m
        x += dt * v
        E, F = force_fn(x)
        v += 0.5 * dt * ACC_UNIT * F / m
        energies.append((E, 0.5 * np.sum(m * v * v) / ACC_UNIT))
    return x, v, energies


def philox_block(seed, step, atom):
    """The four 64-bit words of Philox4x64-10 for counter (atom + 1, step, 0, 0)
    and key (seed, 0).  numpy's generator advances its counter before each
    block, so it is started one below."""
    bg = np.random.Philox(counter=np.array([atom, step, 0, 0], dtype=np.uint64),
                          key=np.array([seed, 0], dtype=np.uint64))
    return bg.random_raw(4)


def gaussian_triplet(seed, step, atom):
    w = philox_block(seed, step, atom)
    u = ((w >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0 ** -24
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    return np.array([r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]), r2 * np.cos(2 * np.pi * u[3])])


def langevin_noise(seed, step, n_atoms):
    return np.stack([gaussian_triplet(seed, step, a) for a in range(n_atoms)]) if n_atoms else np.zeros((0, 3))


def langevin_baoab(pos, vel, masses, force_fn, dt, n_steps, temperature, friction, seed, first_step=0):
    """BAOAB in float64; friction gamma in 1/ps, temperature in K.  Returns
    positions, velocities and (E_pot, E_kin) per step (step 0 first)."""
    x = np.asarray(pos, dtype=np.float64).copy()
    v = np.asarray(vel, dtype=np.float64).copy()
    m = np.asarray(masses, dtype=np.float64)[:, None]
    c1 = np.exp(-friction * 1e-3 * dt)
    c2 = np.sqrt(1.0 - c1 * c1)
    sigma = np.sqrt(KB_EV * temperature * ACC_UNIT / m)          # A/fs, per atom
    E, F = force_fn(x)
    energies = [(E, 0.5 * np.sum(m * v * v) / ACC_UNIT)]
    for s in range(first_step, first_step + n_steps):
        v += 0.5 * dt * ACC_UNIT * F / m
        x += 0.5 * dt * v
        v = c1 * v + c2 * sigma * langevin_noise(seed, s, x.shape[0])
        x += 0.5 * dt * v
        E, F = force_fn(x)
        v += 0.5 * dt * ACC_UNIT * F / m
        energies.append((E, 0.5 * np.sum(m * v * v) / ACC_UNIT))
    return x, v, energies
