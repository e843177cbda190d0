"""Chromatic polynomials of square- and triangular-lattice strips on MI355X.

The hot path (state ranking, per-site factor maps, HIP kernels, runtime) is
native code in ``csrc/`` behind a C ABI (``include/chromstrip.h``); this
package only marshals arguments to it.  Submodules are imported on demand so
that the seeded input generator (``workloads``) can be used without loading
the native library.
"""
