"""MI355X-native Householder Hessenberg-triangular reduction (HouseHT).

The reduction itself runs in the HIP library ``libhtred.so`` (C ABI declared
in ``include/htred.h``); ``paper_1710_08538_amd.htred`` is the thin ctypes
binding over it.  Importing this package does not load the library; the
binding loads it on first use and raises if it is missing.
"""
