"""Parameters of the sampler and the MEGB (oracle's own copy)."""
import dataclasses


@dataclasses.dataclass
class OracleParams:
    n_iters: int = 50        # alternating-projection iterations per trajectory
    n_gn: int = 2            # Gauss-Newton steps per refit (2D-3D)
    n_bis: int = 16          # bisection steps of the pull-in
    megb_iters: int = 4096   # geodesic gradient-descent steps of the MEGB
    megb_avg: int = 10       # iterates averaged for the centre
    omega0: float = 0.5      # initial angular offset magnitude (rad)
    v0: float = 0.2          # initial centre offset magnitude (m)
    kappa: float = 0.999     # projection shrink factor
    tau_abs_3d: float = 1e-5  # feasibility tolerance, metres
    tau_abs_2d: float = 1e-4  # feasibility tolerance, Lambda-units
    z_min: float = 1e-3      # minimum depth (m) for a valid 2D-3D pose
    ckpt_every: int = 5      # checkpoint spacing of the adjoint recompute
    centre_gn: int = 50      # cap on the Gauss-Newton steps of the 2D-3D centre fit
    centre_tol: float = 1e-13  # its convergence test on the step
