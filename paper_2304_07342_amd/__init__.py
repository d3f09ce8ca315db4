"""gpulz: chunked multi-byte LZSS (gpuLZ, ICS'23) on AMD MI355X.

The HIP library (libgpulz.so) is loaded lazily by :mod:`.gpulz`; importing
the package needs neither a GPU nor the built library.
"""
