"""cn: an MI355X-native engine for the fixed-step cable equation over many multi-compartment neurons (the
per-time-step engine of CoreNEURON, arXiv 1901.10975).

Submodules: ``synth`` (seeded synthetic networks), ``cn`` (binding of the HIP library libcn.so), ``build``
(compiles libcn.so for gfx950). Importing the package loads nothing native; ``cn.Engine`` loads libcn.so and fails
loudly when it is missing.
"""
