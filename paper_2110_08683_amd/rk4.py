"""The five-stage, 4th-order SSP-RK time integrator of eqs. (rk4) and
(rk4_substeps) on a single-problem context (GPMood), every stage with its own MOOD
loop.  Each stage runs in the library's kernels (gpm_stage_coef; the state
combination W of the last stage in gpm_lincomb4); this module only sequences them.

Every sub-step U(i) = alpha_i U^n + beta_i U(i-1) - gamma_i dt F(U(i-1)) is the
general stage U_out = a B + b (U_s - cf dt F(U_s)) with a = alpha_i, b = beta_i,
cf = gamma_i / beta_i.  The last combination is read with both dt F terms
subtracted (the printed "+" on the U(3) term is not 4th order):
U^{n+1} = W + b5 (U(4) - cf5 dt F(U(4))), W = c2 U(2) + c3 U(3) - d3 dt F(U(3)),
where dt F(U(3)) = (beta_4 U(3) + alpha_4 U^n - U(4)) / gamma_4 by sub-step 4.
"""
from __future__ import annotations

import torch

# eq. (rk4_substeps): U(i) = ALPHA[i] U^n + BETA[i] U(i-1) - GAMMA[i] dt F(U(i-1))
ALPHA = (0.0, 0.444370493651235, 0.620101851488403, 0.178079954393132)
BETA = (1.0, 0.555629506348765, 0.379898148511597, 0.821920045606868)
GAMMA = (0.391752226571890, 0.368410593050371, 0.251891774271694, 0.544974750228521)
# eq. (rk4): U^{n+1} = C2 U(2) + C3 U(3) - D3 dt F(U(3)) + B5 U(4) - D4 dt F(U(4))
C2, C3, D3 = 0.517231671970585, 0.096059710526147, 0.063692468666290
B5, D4 = 0.386708617503269, 0.226007483236906


def stages():
    """(a, b, cf) of the four sub-steps, the weights of W on (U(2), U(3), U(4), U^n)
    and (a, b, cf) of the last stage."""
    sub = [(ALPHA[i], BETA[i], GAMMA[i] / BETA[i]) for i in range(4)]
    w = (C2, C3 - D3 * BETA[3] / GAMMA[3], D3 / GAMMA[3], -D3 * ALPHA[3] / GAMMA[3])
    return sub, w, (1.0, B5, D4 / B5)


def step(g, U, dt):
    """One SSP-RK4 step of context g from the device tensor U (4, ny, nx) with the
    fixed time step dt; returns U^{n+1} (a new tensor)."""
    sub, w, last = stages()
    g.gpm_set_dt(dt)
    keep = []
    Ui = U
    for a, b, cf in sub:
        out = torch.empty_like(U)
        g.gpm_stage_coef(U if a != 0.0 else None, Ui, out, a, b, cf)
        keep.append(out)
        Ui = out
    W = torch.empty_like(U)
    g.gpm_lincomb4(W, keep[1], w[0], keep[2], w[1], keep[3], w[2], U, w[3])
    out = torch.empty_like(U)
    g.gpm_stage_coef(W, keep[3], out, last[0], last[1], last[2])
    return out
