"""Correctness oracle for the Walsh-Fourier CLS hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only `tests/`, the smoke check in
`__graft_entry__.py` and the CPU-baseline leg of `bench.py` may import, call,
link or execute anything in this package.  It shares no code with the HIP path
and never imports it.

- `coeffs`: exact spectra and Fourier coefficients (eq. wfcoef), Python
  integers and Fractions.
- `native`: FP64 single-threaded C evaluation (ESP recurrence and
  Poisson-binomial routes), projected step, extraction, Philox4x32-10.

Every function is pinned by the `-m "not gpu"` tests against brute force,
closed forms from Appendix A, corner values, multilinearity and published
generator test vectors.
"""
