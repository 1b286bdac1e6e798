"""Physical constants and molecular masses used as *inputs*.

Both the oracle and the HIP library receive these numbers through their
arguments, so the two sides can never disagree on a constant.

Sources: masses of H, He, H2, H2O and CH4 are the values printed in the
paper's mass table (Benchmark section, Table of molecular masses); the other
molecules use standard atomic weights (IUPAC); k_B is exact SI; the atomic
mass unit is CODATA 2018; the Jupiter radius is the paper's value (retrieval
benchmark section); GM_Jup and R_Sun are IAU 2015 nominal values.
"""

K_BOLTZMANN = 1.380649e-23          # J K^-1 (exact SI)
AMU_KG = 1.66053906660e-27          # kg (CODATA 2018)
R_JUP = 6.9911e7                    # m (paper, retrieval benchmark)
R_SUN = 6.957e8                     # m (IAU 2015 nominal)
GM_JUP = 1.2668653e17               # m^3 s^-2 (IAU 2015 nominal)
HE_H2_RATIO = 0.17                  # He/H2 fill ratio (paper, input example)

CONST = {
    "k_B": K_BOLTZMANN,
    "amu": AMU_KG,
    "R_jup": R_JUP,
    "R_sun": R_SUN,
    "GM_jup": GM_JUP,
    "he_h2": HE_H2_RATIO,
}

_AW = {"H": 1.00794, "C": 12.0107, "N": 14.0067, "O": 15.9994,
       "S": 32.065, "Ti": 47.867, "V": 50.9415}

MASSES_AMU = {
    # printed in the paper's mass table
    "H": 1.007940,
    "He": 4.002602,
    "H2": 2.01588,
    "H2O": 18.01528,
    "CH4": 16.04276,
    # standard atomic weights
    "CO": _AW["C"] + _AW["O"],
    "CO2": _AW["C"] + 2 * _AW["O"],
    "NH3": _AW["N"] + 3 * _AW["H"],
    "HCN": _AW["H"] + _AW["C"] + _AW["N"],
    "C2H2": 2 * _AW["C"] + 2 * _AW["H"],
    "H2S": 2 * _AW["H"] + _AW["S"],
    "TiO": _AW["Ti"] + _AW["O"],
    "VO": _AW["V"] + _AW["O"],
}

# Absorber order used by every workload (first n of this list).
ABSORBERS = ["H2O", "CH4", "CO", "CO2", "NH3", "HCN", "C2H2", "H2S", "TiO", "VO"]
