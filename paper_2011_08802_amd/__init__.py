"""MI355X-native Newton-step solver for the finite-strain multivariant
martensite phase-field model (Tuma et al., CMAME 2021).

The product is the C-ABI library ``libmvpf.so`` (``include/mvpf.h``) built from
``csrc/*.hip``; ``mvpf`` is its thin ctypes binding.  Importing this package
does not load the library; ``mvpf.load()`` does, and fails loudly if it has not
been built.
"""
