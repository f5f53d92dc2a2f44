"""MI355X (gfx950) implementation of NeuralVDB's coordinate-MLP encode/decode.

The compute path is the HIP library libnvdb.so (see include/nvdb.h); the
module `nvdb` is its thin ctypes binding.  Import `paper_2208_04448_amd.nvdb`
explicitly: it raises ImportError when the library has not been built.
"""
