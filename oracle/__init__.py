"""Plain FP64 CPU oracle for Kronecker-product exact exchange.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that ``tests/``, the ``smoke()`` check and
the CPU-baseline leg of the benchmark can compare the HIP library against an
obviously correct, slow implementation written directly from the paper.
"""
from .kx_oracle import (  # noqa: F401
    Grid,
    ace_apply,
    ace_apply_complex,
    ace_build,
    ace_build_complex,
    apply_coulomb_multipole,
    apply_fL,
    apply_fL_bloch,
    apply_fL_cell,
    bloch_phases,
    cell_metric,
    derivative_1d_bloch,
    exchange,
    exchange_bloch,
    exchange_cell,
    exchange_multipole,
    fd_weights,
    fd_weights_d1,
    forward_transform,
    kernel_values,
    kernel_values_zero_mode,
    laplacian_1d,
    laplacian_1d_bloch,
    laplacian_cell,
    make_grid,
    make_grid_bloch,
    multipole_moments,
    multipole_potential,
    multipole_rhs_correction,
    node_coords,
    pair_energy,
    pair_potential,
    vx_orbital,
)
