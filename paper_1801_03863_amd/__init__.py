"""MinxEnt-LBM stream-and-collide library for AMD Instinct MI355X (gfx950).

The C ABI is declared in include/lbm.h and implemented by the HIP library
liblbm.so built from csrc/; ``binding`` is its thin Python binding and
``inputs`` draws the seeded synthetic problems.  Modules load lazily so that
the input generators work without the HIP library.
"""
__all__ = ["binding", "inputs", "build"]
