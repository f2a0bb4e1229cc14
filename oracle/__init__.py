"""CPU oracle of the lattice tumour / irradiation simulation (float64, NumPy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the tests, the package smoke check and the
CPU-baseline leg of the benchmark call it.  It shares no code with the HIP
library: both are written from the method's description and meet only in the
tests, on the same seeded inputs.

Modules: philox (Philox4x32-10), model (constants), protocol (validation,
events, LQ thresholds, counting and sampling of protocols), sim (the lattice
automaton), ga (GA operators), ga_slots (the GA over the time-slot genome),
mlp (float64 surrogate network), sga (one generation of the surrogate-screened
GA with a random screen), quasi3d (the variant with several cells per site).
"""
from . import ga, ga_slots, mlp, model, philox, protocol, quasi3d, sga, sim  # noqa: F401
