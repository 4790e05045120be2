"""Pure-Python brute-force evaluations for tiny inputs (pins for the oracle).

Written with scalar ``math`` calls and explicit loops over atoms, pairs and
triplets; it shares no code with ``oracle/``.  Open boundaries only.
"""
import math


def fc(r, rc):
    return 0.5 * math.cos(math.pi * r / rc) + 0.5 if r < rc else 0.0


def pair_index(s, t, ns=7):
    s, t = min(s, t), max(s, t)
    return s * ns - s * (s - 1) // 2 + (t - s)


def aev_brute(pos, species, p):
    """AEV of every atom by O(N^3) loops.  ``p`` is a dict of float params:
    rc_r, eta_r, shf_r, rc_a, eta_a, zeta, shf_a, shf_z, pr, cs."""
    N = len(pos)
    ns = 7
    nr, na, nz = len(p["shf_r"]), len(p["shf_a"]), len(p["shf_z"])
    dim = ns * nr + ns * (ns + 1) // 2 * na * nz
    out = [[0.0] * dim for _ in range(N)]

    def vec(i, j):
        return [pos[j][k] - pos[i][k] for k in range(3)]

    def norm(v):
        return math.sqrt(sum(x * x for x in v))

    for i in range(N):
        for j in range(N):
            if j == i:
                continue
            r = norm(vec(i, j))
            if r >= p["rc_r"]:
                continue
            for k in range(nr):
                out[i][nr * species[j] + k] += p["pr"] * math.exp(-p["eta_r"] * (r - p["shf_r"][k]) ** 2) * fc(r, p["rc_r"])
        for j in range(N):
            for k in range(j + 1, N):
                if j == i or k == i:
                    continue
                vj, vk = vec(i, j), vec(i, k)
                rj, rk = norm(vj), norm(vk)
                if rj >= p["rc_a"] or rk >= p["rc_a"]:
                    continue
                cos_t = sum(a * b for a, b in zip(vj, vk)) / max(rj * rk, 1e-10)
                cos_t = min(1.0, max(-1.0, cos_t))
                theta = math.acos(p["cs"] * cos_t)
                pi = pair_index(species[j], species[k])
                for a in range(na):
                    f2 = math.exp(-p["eta_a"] * ((rj + rk) / 2 - p["shf_a"][a]) ** 2)
                    for z in range(nz):
                        f1 = (0.5 + 0.5 * math.cos(theta - p["shf_z"][z])) ** p["zeta"]
                        col = ns * nr + na * nz * pi + nz * a + z
                        out[i][col] += 2.0 * f1 * f2 * fc(rj, p["rc_a"]) * fc(rk, p["rc_a"])
    return out


def params_of(spec):
    import numpy as np
    f = lambda x: float(np.float32(x))
    return dict(rc_r=f(spec.rc_r), eta_r=f(spec.eta_r), shf_r=[f(x) for x in spec.shf_r],
                rc_a=f(spec.rc_a), eta_a=f(spec.eta_a), zeta=f(spec.zeta),
                shf_a=[f(x) for x in spec.shf_a], shf_z=[f(x) for x in spec.shf_z],
                pr=f(spec.radial_prefactor), cs=f(spec.cos_scale))
