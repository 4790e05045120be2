"""Oracle velocity-Verlet integrator (Sec. 5.4, "Native MD engine": the native
engine reverts to velocity Verlet for NVE dynamics).

    v(t + dt/2) = v(t) + dt/2 a(t)
    x(t + dt)   = x(t) + dt v(t + dt/2)
    v(t + dt)   = v(t + dt/2) + dt/2 a(t + dt),      a = F / m

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
