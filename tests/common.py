"""Helpers shared by the tests: oracle-side reference energies and unit
conversions.  Imports the oracle (test infrastructure) and the input
generator; never the HIP path."""
import numpy as np

import oracle
from paper_1809_07726_amd import synth


def oracle_reference_energies(batch, gb=None):
    """G_ref per (site, state): 0 for state 0 and, for state 1, the change of
    the electrostatic energy of the site's atoms alone (the reference compound)
    at the batch's starting geometry.  An isolated site then titrates exactly
    at pKa_ref / E0_ref."""
    out = np.zeros(2 * batch["n_sites"])
    ms = batch["max_states"]
    for s in range(batch["n_sites"]):
        a, b = batch["site_off"][s], batch["site_off"][s + 1]
        idx = batch["site_atoms"][a:b]
        xyz = batch["xyz"][idx].astype(np.float64)
        _, R, _ = oracle.born(xyz, batch["rho"][idx], batch["screen"][idx], gb)
        q0 = batch["state_q"][a * ms:b * ms].reshape(-1, ms)[:, 0]
        q1 = batch["state_q"][a * ms:b * ms].reshape(-1, ms)[:, 1]
        out[s * ms + 1] = oracle.elec_energy(xyz, q1, R, gb) - oracle.elec_energy(xyz, q0, R, gb)
    return out


def with_oracle_gref(batch, gb=None):
    b = dict(batch)
    b["G_ref"] = oracle_reference_energies(batch, gb)
    return b
