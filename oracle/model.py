"""Model constants of the synthetic tumour / irradiation lattice automaton.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

The paper names the model's ingredients (Materials and Methods, "Underlying
model": diffusion of oxygen, glucose and metabolic waste; cell cycle;
proliferating or quiescent metabolism that responds to local nutrients and pH;
irradiation damage) but defers every equation and constant to earlier work.
The synthetic model used here fixes them as plain inputs.  Field constants are
single-precision values (the GPU state is float32); the oracle converts them to
float64 exactly.  Radiobiology constants are float64.
"""
from dataclasses import dataclass

import numpy as np

EMPTY, PROLIF, QUIESC, DEAD = 0, 1, 2, 3
AGE_MAX = 255
OER_BINS = 16      # oxygen levels of the oxygen effect: bins of O / O_boundary over [0, 1]
DOOM = 1 << 14     # cell-word bit of a lethally hit cell awaiting mitotic death


def _f32(x):
    return float(np.float32(x))


@dataclass
class Params:
    lam: tuple        # FTCS diffusion numbers D*dtau/h^2 for (O, G, H); each <= 1/4
    kappa: tuple      # uptake of O, G and production of H per sub-step at activity 1
    ghost: tuple      # Dirichlet values outside the lattice for (O, G, H)
    init: tuple       # initial uniform field values
    act: tuple        # activity per state (EMPTY, PROLIF, QUIESC, DEAD)
    th_Oq: float      # quiescence below this oxygen
    th_Gq: float      # quiescence below this glucose
    th_Od: float      # necrosis below this oxygen
    th_Gd: float      # necrosis below this glucose
    th_Hd: float      # necrosis above this acidity
    T_min: int        # minimum cycle age (h) before division
    P_div: float      # hourly division probability once T_min is reached
    T_lys: int        # hours from death to lysis (site becomes free)
    A0: int           # initial ages uniform over 0..A0-1
    seed_radius: int  # initial spheroid: (x-c)^2 + (y-c)^2 <= r^2, c = L // 2
    alpha: float      # LQ alpha (1/Gy)
    beta: float       # LQ beta (1/Gy^2)
    class_age: tuple  # proliferating sensitivity classes: age < a0, < a1, >= a1
    m: tuple          # dose multipliers for the classes young, mid, old, quiescent
    repair_half_time: float = 0.0   # hours; 0: sublethal damage repaired between fractions
    oer_max: float = 1.0            # oxygen enhancement ratio at full oxygenation; 1: no oxygen effect
    oer_k: float = 0.05             # oxygen level of half the effect, in the oxygen field's units
    mitotic_death: int = 0          # 1: a lethally hit cell dies at its next division instead of at once

    @classmethod
    def from_dict(cls, d):
        f3 = lambda k: tuple(_f32(v) for v in d[k])
        return cls(
            lam=f3("lambda"), kappa=f3("kappa"), ghost=f3("ghost"), init=f3("init_fields"),
            act=tuple(_f32(v) for v in d["activity"]),
            th_Oq=_f32(d["theta_O_quiesce"]), th_Gq=_f32(d["theta_G_quiesce"]),
            th_Od=_f32(d["theta_O_death"]), th_Gd=_f32(d["theta_G_death"]),
            th_Hd=_f32(d["theta_H_death"]),
            T_min=int(d["T_min"]), P_div=float(d["P_div"]), T_lys=int(d["T_lys"]),
            A0=int(d["A0"]), seed_radius=int(d["seed_radius"]),
            alpha=float(d["alpha"]), beta=float(d["beta"]),
            class_age=tuple(int(v) for v in d["class_age"]),
            m=tuple(float(v) for v in d["m"]),
            repair_half_time=float(d.get("repair_half_time", 0.0)),
            oer_max=float(d.get("oer_max", 1.0)), oer_k=float(d.get("oer_k", 0.05)),
            mitotic_death=int(d.get("mitotic_death", 0)),
        )

    @property
    def oxygen_effect(self):
        return self.oer_max > 1.0

    @property
    def T_div(self):
        """32-bit division threshold: ready iff w3 < T_div = floor(P_div * 2**32)."""
        return min(int(np.floor(self.P_div * 4294967296.0)), 0xFFFFFFFF)
