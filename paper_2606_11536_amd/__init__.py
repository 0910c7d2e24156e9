"""MI355X-native hot path of single-server RLWE PIR: the first-dimension
database scan and the negacyclic NTT/INTT around it (libpir, HIP for gfx950),
with a thin ctypes binding in ``pir``."""

__all__ = ["pir"]
