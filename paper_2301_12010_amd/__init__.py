"""MI355X-native explicit shallow-water step (WENO5 + Lax-Friedrichs flux
splitting + bed/Manning sources + TVD-RK3) after Madden, Marras & Suckale,
arXiv 2301.12010.

``swe`` binds the HIP library ``libswe.so`` (C ABI in ``include/swe.h``);
``inputs`` builds seeded synthetic workloads.  The library is loaded on first
use and its absence is an error.
"""
__all__ = ["swe", "inputs"]
