"""Algorithmic FP64 operation count of one interface of the characteristic
WENO5 sweep, as formulated in ``csrc/ww_sweep.hip``.

Convention: an add, multiply, min/max or compare-select is 1 flop, a fused
multiply-add is 2, a division or square root is 1 (they take several VALU
instructions, so a fraction of peak computed with this count understates the
VALU occupancy).  The count follows the kernel's steps; it is the figure the
benchmark divides by the measured kernel time.
"""

# per-step counts for one interface i+1/2
STEPS = {
    # six stencil cells: velocities (3), total pressure (7), physical flux (24),
    # |lambda^s| for seven fields (6) and their running maxima (7)
    "cell fluxes and LF speeds (6 cells x 47)": 6 * 47,
    # central combination (-F1 + 7F2 + 7F3 - F4)/12 of 7 components (42) and
    # the 5 differences of F and U (70)
    "central term and differences": 42 + 70,
    # mean state (22), sound/Alfven/fast/slow speeds and Roe-Balsara
    # normalisation (53), row/column coefficients (30)
    "interface state and eigen-system": 105,
    "divisions and square roots of the eigen-system": 5 + 8,
    # dW/dU applied to 11 vectors (central term, 5 flux and 5 state
    # differences): 4 x 3 + 14 flops, plus the rotation onto (beta, perp): 12
    "primitive transform of 11 vectors (11 x 35)": 11 * 35,
    # projections onto the 7 left eigenvectors: fast and slow pairs
    # (6 per vector + 22 sign combinations), Alfven (2 per vector + 22),
    # entropy (2 per vector)
    "characteristic projections": 88 + 88 + 44 + 22,
    # per field: LF split of 5 differences on both sides as fused
    # multiply-adds (20), two phi_N (smoothness indicators as expanded
    # quadratic forms 22, squares 3, weights over one denominator 9,
    # interpolant 12 = 46 each), eq. (1) combination (2)
    "WENO5 weights and fluxes (7 fields x 114)": 7 * 114,
    "WENO5 divisions (7 fields x 2)": 14,
    # back-projection: pair sums/differences and primitive columns (31),
    # rotation back (12), dU/dW (23)
    "back-projection": 31 + 12 + 23,
}


def flops_per_interface() -> int:
    return int(sum(STEPS.values()))


if __name__ == "__main__":
    for k, v in STEPS.items():
        print(f"{v:6d}  {k}")
    print(f"{flops_per_interface():6d}  total per interface")


# The textbook formulation of the same interface (dense 7x7 left and right
# eigenvector products on 12 projected vectors, the mean state, the LF split,
# the weights and the back-projection), about 2.35 kflop: a second yardstick
# for the sweep's fraction of peak that does not credit the sparse
# primitive-variable rows.
DENSE_FLOPS_PER_INTERFACE = 2350


RK4_ARRAYS_PER_STAGE = 13 / 4     # RK4 stage forms: 3, 4, 4, 2 arrays read or written


def update_bytes_per_cell(esize: int, integrator: str = "rk4", fused_x: bool = False) -> float:
    """Algorithmic HBM bytes per interior cell of one launch of the flux
    difference / CT / RK update, averaged over the stage forms of a step:
    the 7 stored face components of the three sweeps (one face per cell and
    direction) and the RK arrays: RK4 stages read u0 and write acc, out;
    read u0, acc and write acc, out (twice); read acc and write out
    (3, 4, 4, 2 arrays: 13/4 on average).  fused_x: the update of B only
    (constrained transport; rho, m, E are updated by the fused x sweep):
    the two transverse-B face components of each direction and the three B
    variables of the RK arrays."""
    arrays = {"rk4": RK4_ARRAYS_PER_STAGE, "ssprk3": (2 + 3 + 3) / 3}[integrator]
    if fused_x:
        return 2 * 3 * esize + arrays * 3 * esize
    return 7 * 3 * esize + arrays * 8 * esize


def fused_x_bytes_per_cell(esize: int) -> float:
    """Algorithmic HBM bytes per interior cell of one launch of the x sweep
    with the rho, m, E update fused in, averaged over the RK4 stage forms:
    the state read once (8 variables), the two transverse-B components of
    its x faces written (one face per cell), the y and z faces' rho, m, E
    fluxes read once (5 components, one face per cell and direction), and
    the RK arrays of the five hydro variables."""
    return 8 * esize + 2 * esize + 2 * 5 * esize + RK4_ARRAYS_PER_STAGE * 5 * esize
