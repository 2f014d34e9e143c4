"""Problem description for the oracle (Sec. 1 Eq. conservation laws; Sec. 2.1; Sec. 3.1).

A problem is one of the paper's conservation laws on a uniform Cartesian mesh
(line elements in 1D, squares in 2D: the affine/bilinear maps of Sec. 3.1
reduce to x = x_c + (dx/2) r with Jacobian J = dx/2), with i.i.d. U(-1, 1)
random inputs.  Fields mirror the configuration dictionaries of the shared
input module; nothing here computes any part of the method.
"""

from dataclasses import dataclass, field
from typing import List

NSTATE = {"advection": 1, "burgers": 1, "euler1d": 3, "euler2d": 4}


@dataclass
class Problem:
    equation: str
    nx: int
    p: int
    gpc_order: int
    nq1d: int
    ny: int = 1
    xlo: float = 0.0
    xhi: float = 1.0
    ylo: float = 0.0
    yhi: float = 1.0
    rdim: int = 1
    bc: List[str] = field(default_factory=lambda: ["periodic"] * 4)
    bc_state: List[List[float]] = field(default_factory=lambda: [[0.0] * 4 for _ in range(4)])
    adv_speed: float = 1.0
    gamma: float = 1.4
    flux: str = "rusanov"
    integrator: str = "ssprk3"
    filter: str = "none"
    alpha: float = 36.0
    s: float = 8.0
    nstar: float = 0.0
    eps1: float = 0.6
    eps2: float = 0.6
    sensor: str = "detector"
    s0: float = -1.0
    kappa: float = 4.0
    limiter: bool = False
    cfl: float = 0.3
    t_end: float = 0.0
    # "quad": the nx x ny Cartesian mesh; "tri": the triangle mesh `mesh`
    # (dict of xy [E, 3, 2], nbr [E, 3], nbr_face [E, 3], as made by the shared
    # input module), 2D Euler only
    element: str = "quad"
    mesh: dict = None

    @property
    def dim(self):
        return 2 if self.equation == "euler2d" else 1

    @property
    def S(self):
        return NSTATE[self.equation]

    @property
    def E(self):
        if self.element == "tri":
            return len(self.mesh["xy"])
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def nsp(self):
        if self.element == "tri":
            return (self.p + 1) * (self.p + 2) // 2
        return (self.p + 1) ** self.dim

    @property
    def dx(self):
        return (self.xhi - self.xlo) / self.nx

    @property
    def dy(self):
        return (self.yhi - self.ylo) / self.ny

    @classmethod
    def from_config(cls, cfg):
        keys = cls.__dataclass_fields__.keys()
        return cls(**{k: v for k, v in cfg.items() if k in keys})
