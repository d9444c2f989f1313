"""FP64 CPU oracle for the staggered-grid P_N time step (StaRMAP).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never
does, and it shares no code with the HIP path.

Modules
  basis    real spherical harmonics, flux matrices M_x, M_y, M_z by quadrature,
           sub-grid families by reflection parity          (Sec. 2, eq. (3))
  stepper  literal numpy time stepping: staggered differences, exact
           exponential substep, Strang splitting            (Sec. 2.1, eq. (4)-(6))
  dense    dense/sparse step matrices and Fourier-mode symbols (tiny grids)
  adjoint  transposed step and gradients w.r.t. sigma_a, sigma_s
  c_oracle plain C/OpenMP FP64 implementation of the same literal step for
           full-size configurations (loaded through ctypes)
"""
