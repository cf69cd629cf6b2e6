"""Pin of the oracle against a textbook special case: away from the source,
in a medium with mus' >> mua, Monte Carlo fluence approaches the diffusion
solution.  The reference is the time-resolved extrapolated-boundary dipole
for a semi-infinite medium (Patterson, Chance and Wilson 1989; Farrell,
Patterson and Wilson 1992), integrated over the simulated 0-5 ns window:

    Phi(rho, z, t) = v (4 pi D v t)^-3/2 exp(-mua v t)
                     [exp(-r1^2 / 4Dvt) - exp(-r2^2 / 4Dvt)],
    r1^2 = rho^2 + (z - z0)^2, r2^2 = rho^2 + (z + z0 + 2 zb)^2,
    D = 1/(3(mua + mus')), z0 = 1/mus', zb = 2D (index-matched exit).

Two media with the same mus' (g = 0.01, mus = 1 and g = 0.75, mus = 4) must
both match it, which also pins the use of the anisotropy in the loop.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1711_03244_amd import workloads as W

C = 299.792458


def dipole_fluence(rho, z, mua, musp, n, tmax):
    D = 1 / (3 * (mua + musp))
    v = C / n
    z0 = 1 / musp
    zb = 2 * D
    r1 = rho ** 2 + (z - z0) ** 2
    r2 = rho ** 2 + (z + z0 + 2 * zb) ** 2

    def phi(t):
        if t <= 0:
            return 0.0
        q = 4 * D * v * t
        return v * (math.pi * q) ** -1.5 * math.exp(-mua * v * t) * (
            math.exp(-r1 / q) - math.exp(-r2 / q))

    val, _ = integrate.quad(phi, 0, tmax, limit=200, points=[1e-3, 1e-2, 0.1, 1.0])
    return val


@pytest.mark.parametrize("mus,g,N", [(1.0, 0.01, 1_000_000), (4.0, 0.75, 300_000)])
def test_fluence_matches_diffusion_dipole(oracle_mod, mus, g, N):
    p = W.with_medium(W.cube_homogeneous(), 1, (0.005, mus, g, 1.37))
    mua, mus_, g_, n = (float(x) for x in p.media[1])
    r = oracle_mod.run(p, N, seed=77, nthreads=8)
    phi = oracle_mod.normalise(r["tally"], N, p.h, p.dt, kind=1)[0]
    c = np.arange(60) + 0.5
    yy, xx = np.meshgrid(c, c, indexing="ij")
    rho = np.hypot(xx - p.src_pos[0], yy - p.src_pos[1])
    sel = rho <= 2.5                      # 21 voxels around the beam axis
    depths = [10, 15, 20, 25, 30]
    mc, th = [], []
    for k in depths:
        mc.append(phi[k][sel].mean())
        th.append(np.mean([dipole_fluence(rr, c[k], mua, mus_ * (1 - g_), n, p.ngates * p.dt)
                           for rr in rho[sel]]))
    mc, th = np.array(mc), np.array(th)
    assert np.all(np.abs(mc / th - 1) < 0.10), mc / th
    slope_mc = np.polyfit(c[depths], np.log(mc), 1)[0]
    slope_th = np.polyfit(c[depths], np.log(th), 1)[0]
    assert abs(slope_mc / slope_th - 1) < 0.05, (slope_mc, slope_th)
