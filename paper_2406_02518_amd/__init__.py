"""MI355X-native DDGS-CT DRR splatting renderer (arXiv 2406.02518).

The compute path lives in ``libddgs.so`` (HIP kernels for gfx950 behind a C
ABI, declared in ``include/ddgs.h``).  ``binding`` marshals arguments to it;
``autograd`` wraps render/backward in a ``torch.autograd.Function``;
``synth`` draws seeded synthetic inputs.  Importing the package loads nothing;
``binding.lib()`` raises if the HIP library has not been built.
"""
__all__ = ["binding", "autograd", "synth"]
