"""MI355X-native stereo-LiDAR SGM (census + DDC, semidensification,
multi-path SGM, WTA + subpixel, stereo-LiDAR consistency check).

The compute path is the HIP library ``libsldf.so`` built from ``csrc/``;
``sldf`` is its thin ctypes binding.  Importing the package loads nothing;
the library is loaded on first use and its absence is an error.
"""
