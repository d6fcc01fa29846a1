"""Plain FP64 CPU oracle for the FC(Gram)-based spectral ISPH step.

This package is TEST INFRASTRUCTURE. It exists only to check the GPU library
against a slow, obviously correct implementation written from the paper
(Lin, Fourtakas & Rogers, "A high-order Fourier Continuation (FC)-based
spectral incompressible SPH scheme ...").  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import it.
The product path (``paper_2606_06247_amd``) never imports, links or runs
anything here, and nothing here imports the product path.

Modules
-------
fcgram     FC(Gram) matching/continuation matrices in extended precision
           (Sec. "Fourier Continuation (FC) Algorithm", FC(Gram) paragraph;
           Neumann row from eq. FCNeumann).
fc         FC apply along walled axes (eqs. eq:fc_extended, eq:fc_2d).
kernels    Wendland C2 kernel closed forms and lattice taps.
operators  SPH gradient / divergence / Laplacian as the circular convolution
           of eq. circularConv, evaluated as a direct tap sum (no FFT), plus an
           FFT mode (scipy.fft) of the same math used only for CPU timing.
ppe        Spectral pressure-Poisson solve by dense per-axis transforms
           (eqs. DCTI4PPE, DCTDFT_PPE, division4PPE).
step       One first-order projection step (eqs. uStarRK3, rhsMomtem, PPE,
           u^n+1 with the first-order coefficients a = g = 1, z = 0).
lattice    Lattice geometry shared by the modules above.

Parity status of every function is listed in each module header.
"""
