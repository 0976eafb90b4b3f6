"""Physical constants (CODATA 2018) used by the oracle."""

ALPHA_FS = 7.2973525693e-3          # fine-structure constant
HBAR_C_EV_NM = 197.3269804          # hbar*c in eV nm
ME_C2_KEV = 510.99895000            # electron rest energy in keV
