"""Diagnostics of Sec. 4: effective resolution, Courant numbers, error norms.

H = min diam(K); C = r c dt sqrt(d) / H and C_adv = r U dt sqrt(d) / H; discrete
l2 / l_inf errors over sample points and the experimental order of
convergence EOC = log(e2/e1) / log(h2/h1).
"""
import math
import numpy as np


def courant(r, speed, dt, H, d):
    return r * speed * dt * math.sqrt(d) / H


def box_diameter(*h):
    return math.sqrt(sum(x * x for x in h))


def l2_error(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))


def linf_error(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def eoc(e1, e2, h1, h2):
    return math.log(e2 / e1) / math.log(h2 / h1)


def dofs_per_scalar(n_cells, r, d=3):
    return n_cells * (r + 1) ** d
