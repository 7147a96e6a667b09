"""Unit constants used by the oracle (its own copy; the HIP path receives them as arguments).

Units: Angstrom, eV, amu, fs, K.  The paper fixes no units; these are the conventional ones
for the argon/copper systems it benchmarks (Section 4).
"""
# Elementary charge and atomic mass constant, CODATA 2018 (exact / recommended values).
E_CHARGE = 1.602176634e-19  # C
AMU = 1.66053906660e-27  # kg

# 1 eV / (Angstrom * amu) in Angstrom / fs^2:  (e J) / (1e-10 m * u kg) = e/(u) * 1e10 m/s^2,
# and 1 m/s^2 = 1e10 A / (1e30 fs^2) = 1e-20 A/fs^2.
ACCEL_EV_A_AMU = E_CHARGE / AMU * 1e10 * 1e-20

# Boltzmann constant in eV/K: k_B (exact, J/K) / e (exact, C).
K_B = 1.380649e-23 / E_CHARGE

# FIRE time unit: Angstrom * sqrt(amu / eV), in fs.
TAU_FS = 1.0 / ACCEL_EV_A_AMU ** 0.5
