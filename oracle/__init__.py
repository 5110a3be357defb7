"""CPU FP64 oracle for the model-visibility prediction path.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import, call or execute anything here.  It
shares no code with the GPU library (paper_1909_03956_amd) and imports
nothing from it; both are fed by the seeded generators in synth/.

Plain, slow NumPy: the direct sum of Eq. 12, the nested equal-area sphere
pixelisation of section 3.2, the wavelet tree of Eqs. 9, 10, 16, 17, the
exact adjoint of Eq. 12 and the chi^2 gradients.  What pins each part
(tests/test_oracle_*.py, all CPU):

visibility.predict_direct  unit source at the phase centre gives V = 1; a
    shifted source has |V| = 1 and V(B1 + B2) = V(B1) V(B2); w = 0 on a
    regular grid equals numpy's 2-D FFT (Eq. 2); Pythagorean directions with
    integer phases give V = 1 including the w-term; Hermitian symmetry and
    the sign flip; 50-digit mpmath brute force on small random inputs.
visibility.adjoint         <A x, y> = <x, A^H y> for random complex x, y;
    unit source at the centre with y = 1 gives N_vis; FFT special case.
visibility.grad_direct     central finite differences of chi^2; flux
    gradient equals -2/sigma^2 Re(A^H r); zero at the true model.
visibility.residual_chi2   chi^2 of known residuals (closed form).
sphere.*                   (pixels found by descent: base pixel, then the
    child quarter holding the point, level by level) N_j = 12 4^(j-1); the
    twelve base-pixel centres; every centre is a closed-form centre of the
    HEALPix ring scheme; children 0/1/2/3 at the south/east/west/north corner
    of every pixel, every face row, levels 1-29; nested parent rule
    k_j = k_J >> 2(J-j); round trip pix -> centre -> pix; equal areas
    (Monte-Carlo chi^2); frame axes (P -> (alpha_P, delta_P), u east,
    v north); the recommended-resolution table (tests/golden).
clean.*                    (the clean loop) unit-source dirty image and beam;
    Hogbom as a sort (gain 1, delta beam), as a geometric series, and
    model + residual = image; cross reference = the tree builder's pixels;
    clean-beam fit of a sampled Gaussian; Eq. 6 linear and peaked; the loop
    lowers chi^2 and finds pixel-centred sources.
degrid.*                   (the FFT + degridding comparator) error against
    the direct sum falls with the kernel width and stays under 10^(2 - W);
    conjugate under the sign flip; converged quadrature.
tree.*                     analysis followed by synthesis recovers lambda_J;
    uniform model gives gamma = 0; single component gives F eta_leaf; J = 1;
    Eq. 17 equals the snapped direct sum; the unmasked full-sphere tree
    gives the same V (zero branches may be skipped).
"""
from . import clean, degrid, sphere, tree, visibility  # noqa: F401
