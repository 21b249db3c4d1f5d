"""Closed-form initial fields and source waveforms, evaluated at caller-supplied points.

Conventions (dimensionless units with c = 1, as the paper uses after eq. 6):
the plane has coordinates (x1, x2) = (x, z) and unit normal n = x1 x x2; the scalar magnetic
field is B = B.n. A vacuum plane wave travelling along the unit wavevector k^ carries
E = B (n x k^) with B and E in phase, so an edge with unit tangent t sees the projection
E.t = B * (t . (n x k^)), where n x k^ = (-k^_2, k^_1).
"""
import numpy as np


def cavity_mode(O, m, n, Lx=1.0, Ly=1.0):
    """TE(m, n) mode of a closed rectangular resonator: B = cos(m pi x/Lx) cos(n pi z/Ly)."""
    O = np.asarray(O, dtype=np.float64)
    return np.cos(m * np.pi * O[:, 0] / Lx) * np.cos(n * np.pi * O[:, 1] / Ly)


def periodic_wavevector(theta, cells_per_wavelength, h, L=1.0):
    """Wavevector 2*pi*(m1, m2)/L with integers (m1, m2) nearest to the requested wave.

    Returns (k float64[2], realised angle, realised cells per wavelength).
    """
    lam = cells_per_wavelength * h
    m = np.round(np.array([np.cos(theta), np.sin(theta)]) * L / lam)
    if not np.any(m):
        m = np.array([1.0, 0.0])
    k = 2.0 * np.pi * m / L
    kn = float(np.hypot(k[0], k[1]))
    return k, float(np.arctan2(k[1], k[0])), float(2.0 * np.pi / kn / h)


def random_angle(seed):
    return float(np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi))


def _min_image(delta, L, periodic):
    return delta - L * np.round(delta / L) if periodic else delta


def plane_wave_packet(O, C, tangent, k, dt, sigma=None, center=(0.5, 0.5), L=1.0,
                      periodic=True, phase=0.0):
    """Gaussian-enveloped plane wave, consistent between E and B under leap-frog.

    O: [n_t, 2] points where B lives (circumcentres), C: [n_e, 2] edge midpoints,
    tangent: [n_e, 2] unit edge tangents.  B is returned at t = dt/2 and E at t = 0:
        B = env(O) cos(k.O - |k| dt/2 + phase),
        E = env(C) cos(k.C + phase) (t . (n x k^)).
    sigma=None gives an unbounded plane wave (env = 1).
    """
    O = np.asarray(O, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    tangent = np.asarray(tangent, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    kn = float(np.hypot(k[0], k[1]))
    pol = np.array([-k[1], k[0]]) / kn
    cen = np.asarray(center, dtype=np.float64)

    def env(P):
        if sigma is None:
            return np.ones(len(P))
        r = _min_image(P - cen, L, periodic)
        return np.exp(-(r[:, 0] ** 2 + r[:, 1] ** 2) / (2.0 * sigma * sigma))

    B = env(O) * np.cos(O @ k - kn * dt / 2.0 + phase)
    E = env(C) * np.cos(C @ k + phase) * (tangent @ pol)
    return B, E


def source_waveform(t, omega, n_cycles):
    """sin(omega t) sin^2(pi t / T), T = n_cycles * 2 pi / omega, and 0 outside [0, T)."""
    t = np.asarray(t, dtype=np.float64)
    T = n_cycles * 2.0 * np.pi / omega
    g = np.sin(omega * t) * np.sin(np.pi * t / T) ** 2
    return np.where((t >= 0) & (t < T), g, 0.0)
