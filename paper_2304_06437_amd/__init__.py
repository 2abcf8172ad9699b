"""Thread-safe regularized lattice Boltzmann on AMD MI355X (gfx950).

The compute path is the C-ABI library ``liblb.so`` built from ``csrc/``
(hand-written HIP kernels); ``lb`` is its thin ctypes binding.  Importing this
package loads nothing: the library is opened on first use of ``lb``.
"""
