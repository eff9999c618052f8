"""MI355X deconvolution library: G u = ubar on periodic grids (San & Vedula).

The compute path is libgdecon.so (hand-written HIP for gfx950); ``gdecon``
is its ctypes binding.  ``synth`` draws the seeded synthetic input fields.
Submodules are imported lazily so that the input generator can be used on a
machine without the built library.
"""
__all__ = ["gdecon", "synth"]
