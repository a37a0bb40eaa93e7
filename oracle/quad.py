"""Triangle quadrature for the oracle.

The plane-wave load (the incident-field term of the absorbing boundary
condition in the decomposed BVP, Section II) is an oscillatory surface
integral with no closed form used here.  The oracle integrates it with a
Gauss-Legendre product rule on the unit square mapped onto the reference
triangle by the collapsed (Duffy) map s = u, t = (1-u) v, Jacobian (1-u).
With q points per direction the rule integrates every polynomial in (s, t)
of total degree <= 2q-2 exactly (pinned in tests against the closed form
int s^a t^b = a! b! / (a+b+2)!).
"""
import numpy as np


def triangle_rule(q: int = 8):
    """Points (s, t) and weights on the reference triangle {s,t >= 0, s+t <= 1}.

    Weights sum to the reference area 1/2.
    """
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    s = u.ravel()
    t = ((1.0 - u) * v).ravel()
    wt = (wu * wv * (1.0 - u)).ravel()
    return s, t, wt
