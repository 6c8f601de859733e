"""wsx: GPU-resident reinforcement-learning roll-outs on AMD MI355X (gfx950).

The compute path is the C-ABI library built from ``csrc/`` (``libwsx.so``);
``wsx`` is its thin ctypes binding and ``inputs`` draws seeded synthetic
inputs. Importing this package does not load the library.
"""
