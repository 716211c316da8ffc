"""Seeded synthetic inputs handed, unchanged, to both the HIP library and the
oracle.  Random numbers shaped like the workloads (ions uniform in a cylinder
or annulus about the axis, births spread around the pulse's arrival) and
nothing of the method's arithmetic: no field, rate, crossing or push is
computed here."""
import numpy as np

C_LIGHT = 299792458.0


def cylinder_atoms(seed, n, r_max, z_half, r_min=0.0):
    """n positions [m] uniform in area between r_min and r_max, uniform
    azimuth, z uniform in [-z_half, z_half]."""
    rng = np.random.default_rng([int(seed), 0x5EED])
    r = np.sqrt(r_min ** 2 + rng.uniform(size=n) * (r_max ** 2 - r_min ** 2))
    th = rng.uniform(0.0, 2 * np.pi, n)
    z = rng.uniform(-z_half, z_half, n)
    return r * np.cos(th), r * np.sin(th), z


def birth_times(seed, z, slots_per_atom, tau_fwhm, spread=0.8, p_unborn=0.15):
    """slots_per_atom birth times [s] per atom, ascending within the atom, drawn
    around the arrival time z/c with standard deviation spread * tau_fwhm; a
    binomial number of trailing slots per atom is +inf (unborn)."""
    rng = np.random.default_rng([int(seed), 0xB127])
    n, K = len(z), slots_per_atom
    t = np.asarray(z)[:, None] / C_LIGHT + spread * tau_fwhm * rng.normal(size=(n, K))
    t.sort(axis=1)
    born = K - rng.binomial(K, p_unborn, size=n)
    t[np.arange(K)[None, :] >= born[:, None]] = np.inf
    return t.ravel()


def momenta(seed, n, log_spread=8.0):
    """n normalized momenta (u_x, u_y, u_z) with magnitudes spread over
    exp(+-log_spread) and isotropic directions."""
    rng = np.random.default_rng([int(seed), 0x3031])
    return rng.normal(size=(n, 3)) * np.exp(rng.uniform(-log_spread, log_spread, size=(n, 1)))
