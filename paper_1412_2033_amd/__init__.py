"""fftgal: guaranteed bounds on homogenized conductivity (Ga scheme), MI355X-native.

The computation lives in the HIP library built from ``csrc/`` (see ``build.py``);
``fftgal`` is its ctypes binding.  Importing this package loads nothing.
"""
