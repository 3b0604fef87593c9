"""MI355X (gfx950) implementation of the multiple-precision Taylor series
method for the Lorenz system.

The arithmetic runs in the HIP library `libmpts.so` (C ABI in include/mpts.h);
`mpts` is a thin ctypes binding that marshals arguments and hands PyTorch
device memory and streams to it.
"""
