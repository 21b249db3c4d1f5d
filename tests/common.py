"""Shared test helpers: workloads, initial states sampled on each side's own geometry."""
import numpy as np

import meshgen


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def geometry_of(side):
    """(O, C, tangent) from an oracle mesh or a library mesh view dict."""
    if isinstance(side, dict):
        return side["O"], side["C"], side["evec"] / side["elen"][:, None]
    return side.O, side.C, side.tangent


def cavity_state(side):
    O, C, _ = geometry_of(side)
    B = meshgen.cavity_mode(O, 1, 1)
    return np.zeros(len(C)), B


def packet_state(side, dt, n, theta=0.7, cells=20.0, sigma=0.1):
    O, C, t = geometry_of(side)
    k, _, _ = meshgen.periodic_wavevector(theta, cells, 1.0 / n)
    B, E = meshgen.plane_wave_packet(O, C, t, k, dt, sigma=sigma, center=(0.5, 0.5))
    return E, B
