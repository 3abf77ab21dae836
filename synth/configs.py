"""Workload descriptions of the synthetic FSI systems (no arithmetic).

Physics follows the steady Hron-Turek parameter table of the paper (fluid
density 1000, viscosity 1, incompressible neo-Hookean solid with shear
modulus 5e5); the geometry is a straight channel with a rectangular
(box-shaped in 3D) solid obstacle clamped to the bottom wall, which stands in
for the benchmark meshes that are not available.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class ProblemSpec:
    dim: int = 2
    nx: int = 16                 # finest-level elements in x
    ny: int = 4
    nz: int = 1                  # ignored in 2D
    levels: int = 2              # multigrid levels (finest = the given mesh)
    patch: int = 2               # Schwarz patch = patch^dim element box
    lx: float = 4.0
    ly: float = 1.0
    lz: float = 1.0
    solid_lo: tuple = (1.0, 0.0, 0.0)
    solid_hi: tuple = (1.5, 0.5, 1.0)
    rho: float = 1000.0
    mu: float = 1.0
    mu_s: float = 5.0e5
    u_peak: float = 0.2
    amp: float = 0.05            # velocity perturbation amplitude
    pressure: str = "p1disc"     # "p1disc" (the paper's Q2-P1disc) or "q1" (continuous per material)
    seed: int = 1
    # Crank-Nicolson time step (transient): the linearisation is a Newton
    # iterate at t_{n+1} whose displacement differs from the state at t_n by
    # amp_d times the normalised Fourier shape of the velocity perturbation
    transient: bool = False
    dt: float = 0.01             # the paper's FSI3-T-2D time step
    rho_s: float = 1000.0        # solid density
    amp_d: float = 1.0e-3
    # local solves of the fluid blocks: ILU(0) instead of the exact inverse
    fluid_ilu: bool = False
    # solver settings
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.7
    restart: int = 30
    rtol: float = 1e-10
    maxit: int = 1000
    name: str = "custom"

    def with_(self, **kw) -> "ProblemSpec":
        return replace(self, **kw)

    @property
    def coarse_shape(self):
        f = 2 ** (self.levels - 1)
        return (self.nx // f, self.ny // f, max(self.nz // f, 1))


CONFIGS = {
    # 16x4 Q2/Q1, 2 levels, 2x2 patches, FP64, FGMRES(30) to 1e-10
    "c0_2d_16x4": ProblemSpec(dim=2, nx=16, ny=4, levels=2, patch=2, rtol=1e-10,
                              name="2d_16x4_L2_p2"),
    # 128x32, 4 levels (coarsest 16x4), 4x4 patches, FP64
    "c1_2d_128x32": ProblemSpec(dim=2, nx=128, ny=32, levels=4, patch=4, rtol=1e-10,
                                name="2d_128x32_L4_p4"),
    # same system, mixed-precision V-cycle, target true residual 1e-8
    "c2_2d_128x32_mixed": ProblemSpec(dim=2, nx=128, ny=32, levels=4, patch=4, rtol=1e-8,
                                      name="2d_128x32_L4_p4_mixed"),
    # one Crank-Nicolson time step of the 128x32 system and of the 16x4 system
    "c4_2d_128x32_cn": ProblemSpec(dim=2, nx=128, ny=32, levels=4, patch=4, rtol=1e-10, transient=True,
                                   name="2d_128x32_L4_p4_cn"),
    "c5_2d_16x4_cn": ProblemSpec(dim=2, nx=16, ny=4, levels=2, patch=2, rtol=1e-10, transient=True,
                                 name="2d_16x4_L2_p2_cn"),
    # 3D 32x8x8, 3 levels (coarsest 8x2x2), 2x2x2 patches, mixed, rtol 1e-8
    "c3_3d_32x8x8": ProblemSpec(dim=3, nx=32, ny=8, nz=8, levels=3, patch=2, rtol=1e-8,
                                name="3d_32x8x8_L3_p2"),
}


def config(name: str) -> ProblemSpec:
    return CONFIGS[name]
