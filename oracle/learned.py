"""FP64 oracle of the learned coefficient correction (TEST INFRASTRUCTURE ONLY).

The plain method's numerical dispersion comes from the irregular geometry of the mesh (the
paper notes that eq. 3 is most accurate for equilateral triangles, and studies dispersion
in Section 2).  The correction multiplies the coefficients of edge i in eq. 3 and eq. 4 by
gamma_i = 1 + 0.1 tanh(z_i), where z_i is a small MLP of eight local geometry features.  With
both coefficients scaled, metric (7) is still conserved exactly.

Everything here is written from those definitions in plain numpy FP64:
- `features`: the eight per-edge features;
- `mlp_forward` / `mlp_param_grad`: 8 -> 32 -> 32 -> 1 with tanh, and its exact backward;
- `rq_phase_error` / `rq_loss_grad`: phase error of a sampled plane wave from the Rayleigh
  quotient of K_gamma = -L_E L_B (gamma) with the leap-frog correction, and its gradient in
  gamma;
- `timestepped_phase_error`: phase velocity measured by stepping a complex plane wave with the
  oracle stepper (two real runs) and fitting the phase of its overlap with the initial wave.
"""
import numpy as np

N_FEAT, H1, H2 = 8, 32, 32
SIZES = [("W1", (H1, N_FEAT)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("w3", (H2,)),
         ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)      # 1377
GAMMA_SPAN = 0.1


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shape)
        o += n
    return out


def _angle(u, v):
    cross = u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]
    dot = u[:, 0] * v[:, 0] + u[:, 1] * v[:, 1]
    return np.arctan2(np.abs(cross), dot)


def features(om):
    """Eight features per edge, symmetric under swapping R and L and reversing the edge:
    0 d/|e|; 1, 2 min/max of the angles opposite the edge in R and L; 3, 4 min/max of
    circumradius / shortest side of R and L; 5 |hR - hL|/d; 6 |e|/sqrt(mean area);
    7 |S_R - S_L|/(S_R + S_L).  Outer edges use their one triangle twice."""
    ne = om.ne
    P = om.xy[om.tri]                                   # [nt, 3, 2] (winding CCW)
    rel = P - P[:, :1, :]
    if om.periodic:
        rel[..., 0] -= om.Lx * np.round(rel[..., 0] / om.Lx)
        rel[..., 1] -= om.Ly * np.round(rel[..., 1] / om.Ly)
    side = np.stack([np.hypot(*(rel[:, (q + 1) % 3] - rel[:, q]).T) for q in range(3)], 1)
    u = om.O - om.xy[om.tri[:, 0]]
    if om.periodic:
        u[:, 0] -= om.Lx * np.round(u[:, 0] / om.Lx)
        u[:, 1] -= om.Ly * np.round(u[:, 1] / om.Ly)
    circ_r = np.hypot(u[:, 0], u[:, 1])
    rho_t = circ_r / side.min(1)
    # angle opposite local edge q sits at local vertex q+2
    ang = np.zeros((om.nt, 3))
    for q in range(3):
        w = rel[:, (q + 2) % 3]
        ang[:, q] = _angle(rel[:, q] - w, rel[:, (q + 1) % 3] - w)
    # per edge: values of the R and L triangles
    aR = np.zeros(ne); aL = np.zeros(ne)
    for q in range(3):
        i = om.A[:, q]
        isR = om.s[:, q] > 0
        aR[i[isR]] = ang[isR, q]
        aL[i[~isR]] = ang[~isR, q]
    R = np.where(om.R >= 0, om.R, om.L)
    L = np.where(om.L >= 0, om.L, om.R)
    aR = np.where(om.R >= 0, aR, aL)
    aL = np.where(om.L >= 0, aL, aR)
    f = np.zeros((ne, N_FEAT))
    f[:, 0] = om.d / om.elen
    f[:, 1] = np.minimum(aR, aL)
    f[:, 2] = np.maximum(aR, aL)
    f[:, 3] = np.minimum(rho_t[R], rho_t[L])
    f[:, 4] = np.maximum(rho_t[R], rho_t[L])
    f[:, 5] = np.abs(om.hR - om.hL) / om.d
    f[:, 6] = om.elen / np.sqrt(np.mean(om.S))
    f[:, 7] = np.abs(om.S[R] - om.S[L]) / (om.S[R] + om.S[L])
    return f


def mlp_forward(theta, feat, mu, sd, want_cache=False):
    """gamma = 1 + 0.1 tanh(w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3), x = (f - mu)/sd."""
    p = unpack(theta)
    x = (np.asarray(feat, np.float64) - mu) / sd
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    z = h2 @ p["w3"] + p["b3"][0]
    t = np.tanh(z)
    gamma = 1.0 + GAMMA_SPAN * t
    if want_cache:
        return gamma, dict(x=x, h1=h1, h2=h2, t=t)
    return gamma


def mlp_param_grad(theta, feat, mu, sd, dL_dgamma):
    """Gradient of sum_i dL/dgamma_i * gamma_i(theta) with respect to theta (backprop)."""
    p = unpack(theta)
    _, c = mlp_forward(theta, feat, mu, sd, want_cache=True)
    g = np.asarray(dL_dgamma, np.float64) * GAMMA_SPAN * (1.0 - c["t"] ** 2)   # dL/dz
    d2 = g[:, None] * p["w3"][None, :] * (1.0 - c["h2"] ** 2)                   # dL/d(pre2)
    d1 = (d2 @ p["W2"]) * (1.0 - c["h1"] ** 2)                                 # dL/d(pre1)
    grads = {"W1": d1.T @ c["x"], "b1": d1.sum(0), "W2": d2.T @ c["h1"], "b2": d2.sum(0),
             "w3": c["h2"].T @ g, "b3": np.array([g.sum()])}
    return np.concatenate([grads[n].reshape(-1) for n, _ in SIZES])


def rq_terms(om, k):
    """a_i(k) = (|e_i|/d_i) |exp(i k.O_R) - exp(i k.O_L)|^2 on interior edges (0 outside)."""
    k = np.asarray(k, np.float64)
    a = np.zeros(om.ne)
    i = om.interior
    dO = om.O[om.R[i]] - om.O[om.L[i]]
    a[i] = om.elen[i] / om.d[i] * (2.0 - 2.0 * np.cos(dO @ k))
    return a


def rq_phase_error(om, gamma, dt, k):
    """Signed phase-velocity error of the sampled plane wave exp(i k.O) under K_gamma:
    omega_RQ^2 = sum_i gamma_i^2 a_i / sum_j S_j, corrected for leap-frog,
    omega = (2/dt) asin(omega_RQ dt / 2), error = omega/|k| - 1."""
    g = np.ones(om.ne) if gamma is None else np.asarray(gamma, np.float64)
    w2 = np.sum(g * g * rq_terms(om, k)) / np.sum(om.S)
    w = 2.0 / dt * np.arcsin(np.sqrt(w2) * dt / 2.0)
    return w / np.hypot(k[0], k[1]) - 1.0


def rq_loss_grad(om, gamma, dt, waves):
    """Mean squared RQ phase error over `waves` and its gradient in gamma."""
    g = np.asarray(gamma, np.float64)
    A = np.sum(om.S)
    loss, grad = 0.0, np.zeros(om.ne)
    for k in waves:
        a = rq_terms(om, k)
        w_rq = np.sqrt(np.sum(g * g * a) / A)
        kn = np.hypot(k[0], k[1])
        s = w_rq * dt / 2.0
        err = 2.0 / dt * np.arcsin(s) / kn - 1.0
        loss += err * err
        derr_dw = 1.0 / (kn * np.sqrt(1.0 - s * s))            # d err / d omega_RQ
        grad += 2.0 * err * derr_dw * (g * a) / (A * w_rq)      # d omega_RQ / d gamma_i
    n = len(waves)
    return loss / n, grad / n


def timestepped_phase_error(om, gamma, dt, k, nsteps, samples=20):
    """Phase velocity of a complex plane wave B = exp(i k.O), E consistent, advanced by the
    oracle stepper as two real runs; omega from a least-squares fit of the unwrapped phase
    of the overlap z(t) = sum w E conj(E0) + sum S B conj(B0)."""
    k = np.asarray(k, np.float64)
    kn = np.hypot(k[0], k[1])
    pol = np.array([-k[1], k[0]]) / kn
    B0 = np.exp(1j * (om.O @ k - kn * dt / 2.0))
    E0 = np.exp(1j * (om.C @ k)) * (om.tangent @ pol)
    E0 = np.where(om.interior, E0, 0.0)
    w = np.where(om.interior, om.d * om.elen, 0.0)
    runs = [(E0.real.copy(), B0.real.copy()), (E0.imag.copy(), B0.imag.copy())]
    chunk = max(1, nsteps // samples)
    ts, zs = [], []
    for s in range(samples):
        for r in range(2):
            out = om.step(runs[r][0], runs[r][1], dt, chunk, n0=s * chunk, gamma=gamma)
            runs[r] = (out["E"], out["B"])
        E = runs[0][0] + 1j * runs[1][0]
        B = runs[0][1] + 1j * runs[1][1]
        z = np.sum(w * E * np.conj(E0)) + np.sum(om.S * B * np.conj(B0))
        ts.append((s + 1) * chunk * dt)
        zs.append(z)
    phase = np.unwrap(-np.angle(np.array(zs)))
    t = np.array(ts)
    slope = np.polyfit(t, phase, 1)[0]
    return slope / kn - 1.0


def _K_sparse(om, gamma):
    """K_gamma = -L_E L_B as a sparse matrix: (K x)_j = (1/S_j) sum over interior edges of j of
    gamma^2 (|e|/d) (x_j - x_other)."""
    import scipy.sparse as sp
    i = om.interior
    R, Lt = om.R[i], om.L[i]
    g = np.ones(om.ne) if gamma is None else np.asarray(gamma, np.float64)
    w = g[i] ** 2 * om.elen[i] / om.d[i]
    rows = np.concatenate([R, Lt, R, Lt])
    cols = np.concatenate([R, Lt, Lt, R])
    K = sp.csr_matrix((np.concatenate([w, w, -w, -w]), (rows, cols)), shape=(om.nt, om.nt))
    return sp.diags(1.0 / om.S) @ K


def ts_steps(k, dt, phase=2.0):
    """Number of leap-frog steps for the wave to advance about `phase` radians."""
    return max(1, int(round(phase / (np.hypot(k[0], k[1]) * dt))))


def ts_phase_error_grad(om, gamma, dt, k, nsteps):
    """Phase error of a plane wave advanced by leap-frog, and its gradient in gamma.

    In vacuum, eliminating E from the two half-steps gives, for x_n = B^{n+1/2},
        x_{n+1} = (2 - dt^2 K) x_n - x_{n-1}.
    Start from x_{-1} = exp(i(k.O + |k| dt/2)), x_0 = exp(i(k.O - |k| dt/2)) (the exact wave
    at t = -dt/2 and +dt/2), take z_n = sum_j S_j conj(Bhat_j) x_{n,j} with Bhat = exp(i k.O),
    phi = -arg(z_N / z_0) and error = phi/(|k| N dt) - 1.
    Gradient: with v_m the same recurrence from v_{-1} = 0, v_0 = Bhat (Chebyshev polynomials
    of the second kind in (2 - dt^2 K)/2 applied to Bhat), a perturbation dK changes z_N by
    -dt^2 sum_{n<N} v_{N-1-n}^H S dK x_n; for edge i,
        dz_N/dgamma_i = -2 dt^2 gamma_i (|e_i|/d_i) sum_n conj(v_{N-1-n,R} - v_{N-1-n,L})
                                                         (x_{n,R} - x_{n,L}).
    The v sequence is run forward to N and then backwards (the recurrence is reversible)."""
    K = _K_sparse(om, gamma)
    k = np.asarray(k, np.float64)
    kn = np.hypot(k[0], k[1])
    Bh = np.exp(1j * (om.O @ k))
    step = lambda cur, prev: 2.0 * cur - dt * dt * (K @ cur) - prev
    x_prev, x = Bh * np.exp(1j * kn * dt / 2), Bh * np.exp(-1j * kn * dt / 2)
    z0 = np.sum(om.S * np.conj(Bh) * x)
    v_prev, v = np.zeros_like(Bh), Bh.copy()
    for _ in range(nsteps):
        x, x_prev = step(x, x_prev), x
        v, v_prev = step(v, v_prev), v
    zN = np.sum(om.S * np.conj(Bh) * x)
    i = om.interior
    R, Lt = om.R[i], om.L[i]
    acc = np.zeros(int(i.sum()), complex)
    x_prev, x = Bh * np.exp(1j * kn * dt / 2), Bh * np.exp(-1j * kn * dt / 2)
    vb, vb_next = v_prev, v                       # v_{N-1}, v_N
    for _ in range(nsteps):
        acc += np.conj(vb[R] - vb[Lt]) * (x[R] - x[Lt])
        x, x_prev = step(x, x_prev), x
        vb, vb_next = step(vb, vb_next), vb
    g = np.ones(om.ne) if gamma is None else np.asarray(gamma, np.float64)
    dz = np.zeros(om.ne, complex)
    dz[i] = -2.0 * dt * dt * g[i] * om.elen[i] / om.d[i] * acc
    T = kn * nsteps * dt
    err = -np.angle(zN / z0) / T - 1.0
    derr = -np.imag(np.conj(zN) * dz) / np.abs(zN) ** 2 / T
    return err, derr


def ts_loss_grad(om, gamma, dt, waves, phase=2.0):
    """Mean squared time-stepped phase error over `waves` and its gradient in gamma."""
    loss, grad = 0.0, np.zeros(om.ne)
    for k in waves:
        e, de = ts_phase_error_grad(om, gamma, dt, k, ts_steps(k, dt, phase))
        loss += e * e
        grad += 2.0 * e * de
    return loss / len(waves), grad / len(waves)


def stiff_reg_loss_grad(feat, gamma, tau=0.02, beta=1e-3, target=0.9):
    """beta * mean over edges with d/|e| < tau of (gamma - target)^2, and its gradient."""
    g = np.asarray(gamma, np.float64)
    sel = np.asarray(feat)[:, 0] < tau
    n = max(1, int(sel.sum()))
    d = np.where(sel, g - target, 0.0)
    return beta * np.sum(d * d) / n, 2.0 * beta * d / n
