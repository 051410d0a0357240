"""MI355X-native deform-and-query path of InstantAvatar (arXiv 2212.10550).

Submodules are imported lazily: ``synth`` (seeded inputs, numpy only) can be
used without the HIP library; ``lib`` (the C-ABI binding), ``pipeline``
(the training step and the frame), ``batch`` (many poses in one graph),
``rootinit`` (the learned root initialiser) and ``autograd`` (the stages as
torch.autograd.Functions) load ``libia355.so`` and fail loudly when it is
missing.
"""
__all__ = ["synth", "lib", "pipeline", "batch", "rootinit", "autograd"]
