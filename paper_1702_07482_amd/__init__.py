"""MI355X-native trained reaction-diffusion despeckling filter (Feng & Chen, 2017).

Submodules:
  synth     seeded synthetic images, speckle and models (no filter arithmetic)
  tnrd      ctypes binding of the C-ABI HIP library libtnrd.so (imported lazily)
"""
__all__ = ["synth"]
