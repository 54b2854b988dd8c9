"""Closed-form hydrodynamic rates that tests measure the solver and the
oracle against.  Written from the Chapman-Enskog results of Sec. II C and
textbook linear acoustics; no solver code."""


def sound_decay_rate(split, Pr, gamma, nu, D=2):
    """Gamma in |a| ~ exp(-Gamma k^2 t) for a sound wave in D dimensions:
    (nu_L + (gamma - 1) alpha) / 2 with the longitudinal viscosity
    nu_L = (2 - 2/D) nu + zeta, zeta = (2/D - R/C_v) tau_zeta R T, R/C_v =
    gamma - 1 and alpha = nu / Pr.  tau_zeta is the time that relaxes the
    trace of the pressure tensor: the shear time, except in split II with
    Pr > 1, whose quasi-equilibrium takes the trace of the non-equilibrium
    pressure tensor out of f*, so that the trace relaxes in the first, faster
    stage, at the thermal time."""
    tau_zeta = nu / Pr if (split == 2 and Pr > 1) else nu
    zeta = (2.0 / D - (gamma - 1)) * tau_zeta
    return ((2 - 2.0 / D) * nu + zeta + (gamma - 1) * nu / Pr) / 2
