"""CPU FP64 oracle of the AR-OAM model-based inversion (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously correct NumPy/SciPy implementation of what the HIP path
computes, written from the paper (Li, Hofmann et al., "Broadband model-based inversion
enables optoacoustic microscopy beyond the acoustic diffraction limit"):

* `oracle.model`     - sub-element discretisation of the spherical sensor (Eq. 3), the
                       electrical impulse response, the lateral sensitivity cut-off, and
                       the compressed single-scan-position model table (Eq. 1-4 with the
                       translational symmetry of the Methods section on scanning symmetries).
* `oracle.operators` - the matrix-vector products A_s u and A_s^T v (Methods, scanning
                       symmetries) and a brute-force dense A_s on tiny grids (Eq. 2-4).
* `oracle.filters`   - the band-pass FIR applied to signals and model columns before
                       inversion (Results; Methods, in vivo imaging).
* `oracle.solvers`   - LSQR for Tikhonov (Eq. 5-6), FISTA with soft-thresholding for L1
                       (Eq. 5, 7), the power iteration for FISTA's Lipschitz constant, and the
                       residual-correction refinement schedules.

Only `tests/`, `__graft_entry__.smoke()` and `bench.py`'s `cpu_baseline` leg may import
this package.  The product path (`paper_2009_10173_amd`) never imports, links or runs it,
and this package imports nothing from the product path.  It shares no code with the HIP
kernels or their host library.

Parity pins (what fixes each function independently of itself) live in
`tests/test_oracle_*.py`.  Functions without an independent pin are marked there and
listed as "parity unpinned": the footprint rule's radius factor (a model-definition
choice) and the physical fidelity of the point-voxel / Gaussian-EIR reading.
"""
from . import filters, model, operators, solvers  # noqa: F401
