"""FP64 CPU oracle for the Image-GS renderer (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import this
package.  It shares no code with the HIP implementation in ``paper_2407_01866_amd``:

* ``cref``   - ctypes wrapper of ``oracle.c`` (brute-force FP64 render + adjoint, OpenMP);
* ``dense``  - an independent NumPy FP64 evaluation of the same definition for tiny inputs;
* ``fitref`` - NumPy FP64 L1 loss/gradient, PSNR and the Adam step of the fitter;
* ``ssimref`` - NumPy FP64 SSIM map, the L1 + 0.1 SSIM loss and its gradient;
* ``initref`` - NumPy FP64 content-adaptive initialization (Eq. 6), error-guided addition
  (Eq. 7) and the progressive schedule;
* ``decoderef`` - NumPy FP64 point evaluation (random access) and the float16 storage format.
"""
