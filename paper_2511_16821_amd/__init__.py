"""MI355X-native scatter-limited hybrid (Q)MC / DG-S_N transport.

The device library (``libslh.so``, HIP for gfx950) is loaded lazily by
``paper_2511_16821_amd.slh``; importing this package loads nothing.
"""
