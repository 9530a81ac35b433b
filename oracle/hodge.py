"""Surface calculus and the Hodge decomposition (TEST INFRASTRUCTURE ONLY).

Section 2: with the chart derivatives X_u, X_v and the metric g_ij, the
surface gradient of psi is (g^11 psi_u + g^12 psi_v) X_u + (g^21 psi_u +
g^22 psi_v) X_v, and the surface divergence of a tangential F = F_1 X_u +
F_2 X_v is |g|^(-1/2) (d_u(|g|^(1/2) F_1) + d_v(|g|^(1/2) F_2)).  Chart
derivatives of node values differentiate the order-k interpolant on each
patch (the reference element's differentiation matrices), and the chart is
the interpolated one (its stored X_u, X_v).

Harmonic vector fields section: a tangential F splits as
F = grad alpha + n x grad beta + H with H harmonic (div H = 0 and
div(n x H) = 0), where Delta alpha = div F and Delta beta = -div(n x F)
(the paper's second equation writes alpha for beta: taking the divergence of
n x F = n x grad alpha - grad beta + n x H gives -Delta beta), and
H = F - grad alpha - n x grad beta.  On a genus-g surface the harmonic
fields span 2g dimensions.
"""
import numpy as np


def _metric(g):
    Xu, Xv = g.Xup, g.Xvp
    E = (Xu * Xu).sum(-1)
    F = (Xu * Xv).sum(-1)
    G = (Xv * Xv).sum(-1)
    return Xu, Xv, E, F, G, E * G - F * F


def surface_gradient(g, psi):
    """grad_Gamma psi at the nodes, (N, 3), for node values psi (N,)."""
    re = g.re
    p = np.asarray(psi, dtype=float).reshape(g.NP, g.n_p)
    pu = p @ re.Du.T
    pv = p @ re.Dv.T
    Xu, Xv, E, F, G, det = _metric(g)
    a = (G * pu - F * pv) / det
    b = (E * pv - F * pu) / det
    return (a[..., None] * Xu + b[..., None] * Xv).reshape(-1, 3)


def surface_divergence(g, V):
    """div_Gamma of the tangential part of V (N, 3) at the nodes, (N,)."""
    re = g.re
    Vp = np.asarray(V, dtype=float).reshape(g.NP, g.n_p, 3)
    Xu, Xv, E, F, G, det = _metric(g)
    cu = (Vp * Xu).sum(-1)
    cv = (Vp * Xv).sum(-1)
    F1 = (G * cu - F * cv) / det
    F2 = (E * cv - F * cu) / det
    J = np.sqrt(det)
    return (((J * F1) @ re.Du.T + (J * F2) @ re.Dv.T) / J).reshape(-1)


def hodge(g, solve, F):
    """(alpha, beta, H) of the tangential field F (N, 3); solve(f) returns
    the mean-zero solution of Delta_Gamma u = f at the nodes."""
    F = np.asarray(F, dtype=float)
    alpha = solve(surface_divergence(g, F))
    beta = solve(-surface_divergence(g, np.cross(g.n, F)))
    H = F - surface_gradient(g, alpha) - np.cross(g.n, surface_gradient(g, beta))
    return alpha, beta, H
