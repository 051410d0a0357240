"""MI355X-native deform-and-query path of InstantAvatar (arXiv 2212.10550).

Submodules are imported lazily: ``synth`` (seeded inputs, numpy only) can be
used without the HIP library; ``ops`` / ``pipeline`` load ``libia355.so`` and
fail loudly when it is missing.
"""
__all__ = ["synth", "ops", "pipeline", "lib"]
