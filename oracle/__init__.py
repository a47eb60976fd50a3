"""Plain FP64 CPU oracle for the Ga (Galerkin, exact integration) bounds.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path (no kernels, headers, helpers, tables or constants); its only
common dependency is the seeded input generator package ``synth``.

Written from the paper (J. Vondrejc, "Improved guaranteed computable bounds on
homogenized properties of periodic media by Fourier-Galerkin method with exact
integration", arXiv:1412.2033), in the paper's order and notation:

* ``grids``     -- index sets Z_N, grid points x_M^m, DFT matrices F_M
                   (Sec. 3.1, eqs. index_set, grid_points, DFT; Sec. 4.1).
* ``fourier``   -- closed-form Fourier coefficients of rect/tri/circ
                   (Remark anal_Fourier, eq. char_func_Four).
* ``material``  -- Fourier coefficients of inclusion and voxel composites and
                   the double-grid matrix A_M (Lemma integ_eval_VM, eq. MBA_GA;
                   eqs. inclcomp_formula, gridcomp_formula; Remark eval_with_FFT).
* ``ga``        -- discrete projections (Def. discrete_proj), the double-grid
                   matrix-vector product (Algorithm 2), conjugate gradients
                   (Remark CG), energy quadrature and bounds (Def. Ga,
                   Prop. struct_bounds).
* ``dense``     -- route O1: the fully populated Fourier-Galerkin matrix
                   (Lemma FD_matrix_full) solved densely at tiny N.

Every function states the passage it follows.  Pins against values fixed by
the paper and by mathematics live in ``tests/test_oracle_*.py``.  The one
printed worked example (the fly-ash eigenvalues of Sec. 6.5) needs an image
that is not available: that comparison is parity unpinned.
"""
