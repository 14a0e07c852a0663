"""Host-side FP64 analysis of sampled observables (Sec. II.B and II.C).

The device path samples integers (per-sweep records, layer profiles); what
the paper does with them afterwards is a handful of small FP64 formulas,
written out here:

* layer means and the dividing surface (Eqs. 17 and 18) and the contact
  angle of the dividing plane;
* the modified Young equation (Eq. 16) integrated along the surface-field
  path for the angle-dependent interface tension gamma(theta);
* the size-set fits of Eq. 20 for gamma(pi/2) and the line tension
  tau(0, pi/2), and the line-tension balance of Eqs. 21 and 22;
* the free-energy difference of two y boundary conditions from a ladder of
  mean energies in beta (Eq. 19 applied to both systems, Eq. 20).

Integrals use the trapezoid rule in the order the points are given, like the
device-side integration of the surface-field path.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# Eqs. 17 and 18: layer means, dividing surface, contact angle
# ---------------------------------------------------------------------------
def row_magnetisation(profile_sum, count: int, Lz: int) -> np.ndarray:
    """m_{k_x}(y) from a profile accumulated over `count` snapshots: an
    (Lx, Ly) array of sums over z (and over the snapshots) divided by
    count * Lz."""
    p = np.asarray(profile_sum, dtype=np.float64)
    return p / (float(count) * float(Lz))


def layer_means(m_rows) -> np.ndarray:
    """Eq. 17: the mean over y of every layer's row magnetisation."""
    m = np.asarray(m_rows, dtype=np.float64)
    return m.sum(axis=1) / m.shape[1]


def plateau_values(m_rows, fraction: float = 0.1):
    """The constant row magnetisations away from the interface, per layer:
    the means of the ceil(fraction * Ly) largest and smallest row values
    (the + and - plateaus).  Requires each phase to cover at least that
    share of the layer; the rows next to the interface, where the profile
    passes its inflection point, then do not enter."""
    m = np.sort(np.asarray(m_rows, dtype=np.float64), axis=1)
    Ly = m.shape[1]
    k = max(1, int(math.ceil(fraction * Ly)))
    return m[:, Ly - k:].mean(axis=1), m[:, :k].mean(axis=1)


def dividing_surface(m_bar, m_plus, m_minus, Ly: int) -> np.ndarray:
    """Eq. 18 with y+ + y- = Ly: the extent y+ of the + domain in every
    layer, y+ = Ly (m_bar - m-) / (m+ - m-)."""
    m_bar = np.asarray(m_bar, dtype=np.float64)
    m_plus = np.asarray(m_plus, dtype=np.float64)
    m_minus = np.asarray(m_minus, dtype=np.float64)
    return float(Ly) * (m_bar - m_minus) / (m_plus - m_minus)


def contact_angle(y_plus, skip: int = 0):
    """Inclination of the dividing plane: a least-squares line
    y+(x) = a + b x through the layers skip .. Lx-1-skip; the plane meets the
    walls (x = const) at theta = atan2(1, |b|), so theta = pi/2 for an
    interface perpendicular to the walls.  Returns (theta, a, b)."""
    y = np.asarray(y_plus, dtype=np.float64)
    x = np.arange(y.size, dtype=np.float64)
    sel = slice(skip, y.size - skip)
    xs, ys = x[sel], y[sel]
    if xs.size < 2:
        raise ValueError("need at least two layers for the fit")
    xm, ym = xs.mean(), ys.mean()
    b = float(((xs - xm) * (ys - ym)).sum() / ((xs - xm) ** 2).sum())
    a = float(ym - b * xm)
    return math.atan2(1.0, abs(b)), a, b


def contact_angle_from_profile(profile_sum, count: int, Lz: int, fraction: float = 0.1, skip: int = 0,
                               m_plus=None, m_minus=None):
    """Eqs. 17 and 18 end to end: accumulated profile -> theta.  The plateau
    values come from plateau_values unless given (e.g. from films with
    periodic y boundaries in the + and - phases)."""
    m = row_magnetisation(profile_sum, count, Lz)
    mb = layer_means(m)
    if m_plus is None or m_minus is None:
        mp, mm = plateau_values(m, fraction)
        m_plus = mp if m_plus is None else m_plus
        m_minus = mm if m_minus is None else m_minus
    yp = dividing_surface(mb, m_plus, m_minus, m.shape[1])
    theta, a, b = contact_angle(yp, skip)
    return {"theta": theta, "y_plus": yp, "intercept": a, "slope": b, "m_bar": mb,
            "m_plus": np.asarray(m_plus, dtype=np.float64), "m_minus": np.asarray(m_minus, dtype=np.float64)}


# ---------------------------------------------------------------------------
# Eq. 16: gamma(theta) along the surface-field path
# ---------------------------------------------------------------------------
def young_gamma(theta, delta_f1, gamma_90: float) -> np.ndarray:
    """Integrates the modified Young equation gamma cos(theta) -
    gamma'(theta) sin(theta) = delta_f1 along a path of points
    (theta_r, delta_f1_r) that starts at theta = pi/2 (H1 = 0) with
    gamma(pi/2) = gamma_90.  With c = cot(theta) the equation reads
    d(gamma / sin theta) / dc = delta_f1, so
    gamma_r = sin(theta_r) (gamma_90 + integral_0^{c_r} delta_f1 dc),
    the integral taken by the trapezoid rule over the given points."""
    th = np.asarray(theta, dtype=np.float64)
    df = np.asarray(delta_f1, dtype=np.float64)
    if th.shape != df.shape or th.ndim != 1 or th.size < 1:
        raise ValueError("theta and delta_f1 must be 1-d arrays of one length")
    c = np.cos(th) / np.sin(th)
    acc = np.zeros_like(th)
    for r in range(1, th.size):
        acc[r] = acc[r - 1] + 0.5 * (c[r] - c[r - 1]) * (df[r - 1] + df[r])
    return np.sin(th) * (gamma_90 + acc)


def young_angle(delta_f1, gamma: float) -> np.ndarray:
    """Young's equation (Eq. 8) for an isotropic tension: cos theta =
    delta_f1 / gamma."""
    return np.arccos(np.asarray(delta_f1, dtype=np.float64) / gamma)


# ---------------------------------------------------------------------------
# Eq. 20 and Eqs. 21-22: interface and line tensions
# ---------------------------------------------------------------------------
def tension_from_sizes(Lx, delta_F_per_area):
    """Eq. 20 divided by Lz Lx: delta_F / (Lz Lx) = gamma(pi/2) +
    (2 / Lx) tau(0, pi/2).  A least-squares line in 1/Lx through the given
    films gives (gamma(pi/2), tau(0, pi/2))."""
    u = 1.0 / np.asarray(Lx, dtype=np.float64)
    v = np.asarray(delta_F_per_area, dtype=np.float64)
    if u.size < 2:
        raise ValueError("need at least two film thicknesses")
    um, vm = u.mean(), v.mean()
    slope = float(((u - um) * (v - vm)).sum() / ((u - um) ** 2).sum())
    gamma = float(vm - slope * um)
    return gamma, slope / 2.0


def line_tension_shift(Lx, Ly, Lz, theta, gamma_theta, gamma_90, surface_sum, surface_diff, ti_gapbc):
    """Eqs. 21 and 22 solved for the line tension: 2 Lz [tau(H1, theta) -
    tau(0, pi/2)] is what remains of the surface-field integral in the
    inclined-interface film (ti_gapbc = F_int(H1) - F_int(0), the
    thermodynamic integral of Eq. 22) after the interface term
    Lx Lz [gamma(theta)/sin(theta) - gamma(pi/2)], the surface term
    Lz Ly surface_sum with surface_sum = gamma+(|H1|) + gamma+(-|H1|) -
    2 gamma+(0), and the contact-line surface term Lz Lx surface_diff /
    tan(theta) with surface_diff = gamma+(|H1|) - gamma+(-|H1|).  Returns
    tau(H1, theta) - tau(0, pi/2) (arrays broadcast)."""
    th = np.asarray(theta, dtype=np.float64)
    interface = Lx * Lz * (np.asarray(gamma_theta, dtype=np.float64) / np.sin(th) - gamma_90)
    surface = Lz * Ly * np.asarray(surface_sum, dtype=np.float64)
    contact = Lz * Lx * np.asarray(surface_diff, dtype=np.float64) * np.cos(th) / np.sin(th)
    return (np.asarray(ti_gapbc, dtype=np.float64) - interface - surface - contact) / (2.0 * Lz)


# ---------------------------------------------------------------------------
# Eq. 19 for two boundary conditions: delta F = F_APBC - F_PBC
# ---------------------------------------------------------------------------
def beta_integral(beta, u) -> np.ndarray:
    """Eq. 19: the cumulative trapezoid integral of U(beta') d beta' over the
    given ladder (first point = reference beta_0)."""
    b = np.asarray(beta, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(b)
    for r in range(1, b.size):
        out[r] = out[r - 1] + 0.5 * (b[r] - b[r - 1]) * (u[r - 1] + u[r])
    return out


def ground_state_reference(beta0: float, J: float, Lx: int, Lz: int, Ly: int | None = None) -> float:
    """The low-temperature reference of Eq. 19 for an antiperiodic minus a
    periodic film (free x surfaces, no fields): at beta0 J = 10 the free
    energy is close to the ground-state energy U0 (Sec. II.C, after Eq. 19),
    and the antiperiodic ground state differs from the periodic one by one
    flat interface across the film, Lx Lz bonds each 2 J dearer, so
    beta0 delta F(beta0) = beta0 * 2 J Lx Lz.  With Ly given, the
    interface-position entropy is included as well: the antiperiodic ground
    state is 2 Ly-fold degenerate (Ly positions, two orientations), the
    periodic one 2-fold, which lowers beta0 delta F by ln Ly; F = U0 drops
    this term, which is small beside beta0 * 2 J Lx Lz."""
    ref = float(beta0) * 2.0 * float(J) * float(Lx) * float(Lz)
    if Ly is not None:
        ref -= math.log(float(Ly))
    return ref


def delta_free_energy(beta, u_apbc, u_pbc, beta_dF0: float = 0.0) -> np.ndarray:
    """Eq. 20 from Eq. 19 applied to both films: beta delta F(beta) =
    beta_0 delta F(beta_0) + integral_{beta_0}^{beta} (U_APBC - U_PBC) d beta',
    returned as delta F(beta) = F_APBC - F_PBC at every ladder point.  The
    reference difference beta_0 delta F(beta_0) is 0 for a reference in the
    disordered phase (beta_0 < beta_c), where no interface exists, and
    ground_state_reference(beta_0, ...) for the low-temperature reference
    beta_0 J = 10; the ladder may run upwards or downwards from beta_0."""
    b = np.asarray(beta, dtype=np.float64)
    d = np.asarray(u_apbc, dtype=np.float64) - np.asarray(u_pbc, dtype=np.float64)
    return (beta_dF0 + beta_integral(b, d)) / b
