"""MI355X-native event simulator (arXiv 2303.02608): thresholded weighted local
regression turning noisy path-traced frames into DVS events.

The compute path is libesim.so (hand-written HIP for gfx950, C ABI in
``include/esim.h``); :mod:`binding` marshals arguments to it and
:mod:`simulator` runs the frame loop.  :mod:`synth` draws seeded synthetic
clips.  Importing the package does not load the library; the binding raises if
it is not built.
"""
__all__ = ["binding", "simulator", "synth"]
