"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  Holds no arithmetic of the scattering method: only contrast
functions sampled at caller-supplied coordinates and measurement layouts."""
import numpy as np


def gaussian_bumps(xy, nbumps, seed, amp=(0.1, 0.3), width=0.15, centre=0.6, rescale_max=None):
    """q(x) = sum_j a_j exp(-|x - c_j|^2 / w^2) at points xy [n, 2], with
    c_j ~ U[-centre, centre]^2 and a_j ~ U[amp]; optionally rescaled so that
    the maximum over the given points equals rescale_max."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-centre, centre, size=(nbumps, 2))
    a = rng.uniform(amp[0], amp[1], size=nbumps)
    xy = np.asarray(xy, dtype=np.float64)
    q = np.zeros(xy.shape[0])
    for j in range(nbumps):
        d2 = (xy[:, 0] - c[j, 0]) ** 2 + (xy[:, 1] - c[j, 1]) ** 2
        q += a[j] * np.exp(-d2 / width ** 2)
    if rescale_max is not None:
        q *= rescale_max / np.max(q)
    return q


def radial_gaussian(xy, amp, sigma):
    """q(r) = amp exp(-r^2 / sigma^2): a smooth radial contrast whose tail is
    negligible outside r = 5 sigma."""
    xy = np.asarray(xy, dtype=np.float64)
    return amp * np.exp(-(xy[:, 0] ** 2 + xy[:, 1] ** 2) / sigma ** 2)


def sine_coefficients(S, seed, scale=0.3, decay=800.0):
    """c_mn = scale * g_mn * exp(-(m^2 + n^2) / decay), g ~ N(0, 1), m, n = 1..S,
    returned as an [S, S] array (row = x mode m, column = y mode n)."""
    rng = np.random.default_rng(seed)
    m = np.arange(1, S + 1)
    g = rng.standard_normal((S, S))
    return scale * g * np.exp(-(m[:, None] ** 2 + m[None, :] ** 2) / decay)


def equispaced_angles(n):
    """2 pi m / n, m = 0..n-1."""
    return 2.0 * np.pi * np.arange(n) / n


def parity_inputs(xy, M, P, seed, nbumps=5, nsample_u=64, nsample_g=256, nprobe=4):
    """Seeded inputs of one library-vs-oracle parity case at PDE-node
    coordinates xy [npde, 2]:
      q      contrast, `nbumps` bumps (centres U[-0.6, 0.6]^2, amplitudes
             U[0.1, 0.3], width 0.15; seed `seed`);
      dq     perturbation: 3 wide bumps (amplitudes U[0.01, 0.02], width
             0.3; seed + 100) plus 1e-3 N(0, 1) noise per node;
      r      complex N(0, 1) + i N(0, 1) array [M, P] (adjoint input);
      iu     sorted PDE-node indices where total fields are compared;
      ig     sorted PDE-node indices where gradients are compared;
      probes [nprobe, npde] N(0, 1) vectors for gradient dot products."""
    xy = np.asarray(xy, dtype=np.float64)
    npde = xy.shape[0]
    q = gaussian_bumps(xy, nbumps, seed, amp=(0.1, 0.3), width=0.15)
    rng = np.random.default_rng(seed + 200)
    dq = gaussian_bumps(xy, 3, seed + 100, amp=(0.01, 0.02), width=0.3) + 1e-3 * rng.standard_normal(npde)
    r = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    iu = np.sort(rng.choice(npde, size=min(nsample_u, npde), replace=False))
    ig = np.sort(rng.choice(npde, size=min(nsample_g, npde), replace=False))
    probes = rng.standard_normal((nprobe, npde))
    return {"q": q, "dq": dq, "r": r, "iu": iu, "ig": ig, "probes": probes}


def add_noise(u, delta, seed):
    """Noise of the form used for the measured data in the experiments of
    Section 4: for each incident direction (row m of u [M, P]),
    u_m + delta ||u_m|| / ||e_m|| e_m with e_m = e1 + i e2 and e1, e2
    standard normal over the P angles (so ||noise_m|| = delta ||u_m||)."""
    u = np.asarray(u, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    scale = delta * np.linalg.norm(u, axis=-1, keepdims=True) / np.linalg.norm(e, axis=-1, keepdims=True)
    return u + scale * e
