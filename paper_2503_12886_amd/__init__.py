"""MI355X-native batch-parallel differentiable renderer for reduced Gaussian
blendshape avatars (blend -> EWA projection -> tile binning and depth order ->
front-to-back alpha compositing, forward and backward).

The compute path is the C-ABI library ``libgbr.so`` (hand-written gfx950 HIP
kernels); ``paper_2503_12886_amd.gbr`` is its thin ctypes binding.  Importing
this package does not load the library; the first call into it does, and it
raises if the library is missing -- there is no CPU fallback.
"""
__all__ = ["gbr", "synth"]
