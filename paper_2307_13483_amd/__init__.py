"""MI355X-native solver for vibronic dynamics of discrete states in the
electron continuum (Cosicova, Dvorak & Cizek, arXiv:2307.13483).

The compute path is the C-ABI library ``libvdc.so`` (hand-written HIP for
gfx950); ``paper_2307_13483_amd.vdc`` is its thin ctypes binding.  Importing
this package loads nothing; ``vdc`` loads the library on first use and fails
loudly when it is missing.
"""
