"""Brute-force NumPy mini-oracle (test infrastructure only), a second implementation independent of oracle.c.

It evaluates arXiv 2212.09807 eq. (current) with the M -> infinity expectation of the diffusion perturbations
directly point by point: for every segment, every sample point, every (tick, x-bin, y-bin) the point's
truncated-Gaussian cloud can reach, every pixel of the grid and every table tick.  No charge-cell tensor,
no support boxes, no pixel selection, and the normal CDF comes from ``scipy.special.ndtr`` rather than erfc.
Only for tiny inputs (a few segments, a few pixels, short tables).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr


def _recomb(ph, dedx):
    eps = ph.e_field * ph.lar_density
    if ph.recomb_model == 0:
        return ph.birks_ab / (1.0 + ph.birks_kb * dedx / eps)
    xi = ph.box_beta * dedx / eps
    r = math.log(ph.box_alpha + xi) / xi if xi > 0 else -math.inf
    return max(r, 0.0)


def _n_points(dx, dy, dz, step):
    f = np.float32
    L = np.sqrt(f(f(f(dx) * f(dx)) + f(f(dy) * f(dy))) + f(f(dz) * f(dz)), dtype=np.float32)
    q = np.float32(L / f(step))
    return max(1, int(np.ceil(q)))


def _trunc_mass(mean, sigma, nsig, lo, hi):
    if sigma == 0.0:
        return 1.0 if lo <= mean < hi else 0.0
    a = max((lo - mean) / sigma, -nsig)
    b = min((hi - mean) / sigma, nsig)
    if a >= b:
        return 0.0
    return (ndtr(b) - ndtr(a)) / (ndtr(nsig) - ndtr(-nsig))


def waveforms(ph, ro, table, segs, pixels):
    """I[p, n] for the listed tile-local pixel ids, FP64."""
    T, BX, BY = table.shape
    R = table.astype(np.float64)
    b = ro.pitch / ro.n_sub
    out = np.zeros((len(pixels), ro.n_ticks))
    for s in range(segs.n):
        x0, y0, z0, t0 = (float(segs.x0[s]), float(segs.y0[s]), float(segs.z0[s]), float(segs.t0[s]))
        x1, y1, z1, t1 = (float(segs.x1[s]), float(segs.y1[s]), float(segs.z1[s]), float(segs.t1[s]))
        E = float(segs.energy[s])
        L = math.sqrt((x1 - x0) ** 2 + (y1 - y0) ** 2 + (z1 - z0) ** 2)
        dedx = E / L if L > 0 else float(segs.dedx[s])
        qr = _recomb(ph, dedx) * E / ph.w_ion
        tdr = abs(0.5 * (z0 + z1) - ph.z_anode) / ph.v_drift
        qa = qr * math.exp(-tdr / ph.lifetime)
        sx = math.sqrt(2 * ph.d_tran * tdr)
        st = math.sqrt(2 * ph.d_long * tdr) / ph.v_drift
        N = _n_points(segs.x1[s] - segs.x0[s], segs.y1[s] - segs.y0[s], segs.z1[s] - segs.z0[s], ph.sample_step)
        for mu in range(N):
            f = (mu + 0.5) / N
            px, py = x0 + f * (x1 - x0), y0 + f * (y1 - y0)
            pz, pt = z0 + f * (z1 - z0), t0 + f * (t1 - t0)
            ta = pt + abs(pz - ph.z_anode) / ph.v_drift
            span = ph.n_sigma * sx + 2 * b
            us = range(int(math.floor((px - span - ro.x0) / b)), int(math.floor((px + span - ro.x0) / b)) + 1)
            vs = range(int(math.floor((py - span - ro.y0) / b)), int(math.floor((py + span - ro.y0) / b)) + 1)
            tspan = ph.n_sigma * st + 2 * ro.tick
            As = range(int(math.floor((ta - tspan - ro.t_begin) / ro.tick)),
                       int(math.floor((ta + tspan - ro.t_begin) / ro.tick)) + 1)
            fx = {u: _trunc_mass(px, sx, ph.n_sigma, ro.x0 + u * b, ro.x0 + (u + 1) * b) for u in us}
            fy = {v: _trunc_mass(py, sx, ph.n_sigma, ro.y0 + v * b, ro.y0 + (v + 1) * b) for v in vs}
            ft = {a: _trunc_mass(ta, st, ph.n_sigma, ro.t_begin + a * ro.tick, ro.t_begin + (a + 1) * ro.tick)
                  for a in As}
            for qi, pid in enumerate(pixels):
                ix, iy = pid % ro.n_x, pid // ro.n_x
                xc = ro.x0 + (ix + 0.5) * ro.pitch
                yc = ro.y0 + (iy + 0.5) * ro.pitch
                for u in us:
                    if fx[u] == 0.0:
                        continue
                    # bin centre offset from the pixel centre, mirrored into the table quadrant
                    ci = abs(ro.x0 + (u + 0.5) * b - xc) / b - 0.5
                    i = int(round(ci))
                    if i >= BX:
                        continue
                    for v in vs:
                        if fy[v] == 0.0:
                            continue
                        cj = abs(ro.y0 + (v + 0.5) * b - yc) / b - 0.5
                        j = int(round(cj))
                        if j >= BY:
                            continue
                        for a in As:
                            if ft[a] == 0.0:
                                continue
                            w = qa / N * fx[u] * fy[v] * ft[a]
                            for k in range(T):
                                n = a - (T - 1) + k
                                if 0 <= n < ro.n_ticks:
                                    out[qi, n] += w * R[k, i, j]
    return out
