"""MI355X-native lattice Boltzmann stream-collide library.

The compute path is the HIP shared library ``liblbm_mi355x.so`` (C ABI in
``include/lbm.h``); ``paper_2001_11806_amd.lbm`` is its thin ctypes binding and
``paper_2001_11806_amd.autograd`` the ``torch.autograd.Function`` on top.
This package file imports nothing eagerly so that ``inputs`` can be used
without loading the library.
"""

__all__ = ["lbm", "autograd", "inputs"]
