"""MI355X-native Lomb-Scargle periodogram (Gowanlock et al., arXiv 2105.04006).

The compute path is the C-ABI library ``liblsp.so`` built from ``csrc/`` for
gfx950; ``lsp`` is its thin Python binding and ``synth`` draws seeded inputs.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
