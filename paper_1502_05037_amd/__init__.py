"""MI355X-native SARA/SDMM for radio-interferometric imaging.

Importing the package loads nothing native.  ``paper_1502_05037_amd.sarahip``
binds the HIP library (``libsarahip.so``) and raises if it is missing;
``paper_1502_05037_amd.synth`` holds the seeded input generators.
"""
__all__ = ["sarahip", "synth"]
