"""liblabs: MI355X-native batched tabu search and memetic tabu search for
Low Autocorrelation Binary Sequences (arXiv:2504.00987).

The compute path is the HIP library ``liblabs.so`` (C ABI in
``include/liblabs.h``); ``labs`` is its Python front end.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built.
"""
__all__ = ["inputs", "labs", "build"]
