"""MI355X (gfx950) direct Poisson solver on a staggered grid by eigenfunction
expansion (Costa et al., arXiv 2001.05234, Section 2).

The solver is the HIP library ``libcans_poisson.so`` behind the C ABI of
``include/cans_poisson.h``; ``capi`` is its ctypes binding.  Importing this
package loads nothing; ``capi.load()`` loads the library and raises if it
has not been built.
"""
