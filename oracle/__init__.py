"""FP64 CPU oracle for SARA solved by SDMM (test infrastructure only).

This package is the plain, slow reference against which the HIP path is checked.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path; inputs come
from ``paper_1502_05037_amd.synth``, which draws random numbers only.

Modules
-------
kb           Kaiser-Bessel interpolation kernel and its Fourier transform.
measurement  The measurement operator: direct DFT, FP64 NUFFT (numpy, and a variant whose
             interpolation loops are compiled C for millions of visibilities), operator norm.
nufft_c.c    Those compiled loops (plain C + OpenMP, float64); cbuild.py builds and loads them.
wavelets     Daubechies filters, periodic DWT, the SARA dictionary.
prox         Soft threshold, l2-ball projection, positive-orthant projection.
sdmm         SDMM on problem (3), conjugate-gradient x-update, SARA reweighting,
             KKT residuals.
problem      Noise scaling, per-block noise bounds, dirty image.
unet         The warm-start U-Net: layers, forward, gradients, Adam, bfloat16 emulation.
"""
