"""CPU FP64 oracle of the non-singular boundary-integral / Fourier-synthesis method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
GPU library never calls it and shares no code with it; both read their inputs
from ``workloads.py`` only.

Modules (each function cites the passage of the paper it follows):
  mesh    - icosphere surfaces, analytic normals, lumped nodal weights
  bie     - discrete non-singular boundary integral equation (Eq. BRIEF with the
            functions of Appendix A and the S_inf integrals of Appendix B), dense
            LAPACK solve
  field   - closest surface node, non-singular field representation (Eq. BRIEFdmn)
  chief   - interior-point conditions added to the surface rows, solved in the
            least-squares sense (the remedy for fictitious resonances)
  quadratic - six-node quadratic elements on geodesic spheres with Gauss
            quadrature (Sec. III, Sec. IV A: 500 elements / 1002 nodes):
            assembly, direct solve and field
  pulse   - incident pulses (Eq. pulse and others), DFT coefficients, time
            synthesis by inverse FFT (Eq. inverseFourier, Sec. IV)
  series  - closed-form spherical-harmonic series for a soft/hard sphere (pins)
  mlp     - FP64 reference of the frequency surrogate network (forward/backward)
"""
