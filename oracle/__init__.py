"""CPU FP64 oracle for the stochastic-Galerkin (SG) diffusion solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
here, and this package never imports the product.

Everything is plain, slow and explicit: NumPy/SciPy in FP64, assembled sparse
matrices, no fusion and no reordering beyond what each definition states.
Each function cites the passage of the paper (Aulisa, Capodaglio, Ke,
"A computational study of preconditioning techniques for the stochastic
diffusion equation with lognormal coefficient") it follows.

Modules
  pc       index sets J(p) and Hermite triple products          (Sec. 2.2)
  kl       Karhunen-Loeve expansion by a Galerkin procedure      (Sec. 2.1)
  fem      Q1 finite elements, quadrature, stiffness and mass    (Sec. 2.2)
  q2       biquadratic elements: stiffness, mass, the SG system (Sec. 2.2)
  system   coefficient chaos modes, A_k, K = sum G_k (x) A_k, F (Sec. 2.2)
  gmg      geometric multigrid V-cycle on the mean stiffness     (Sec. 3)
  precond  mean-based and field-split block Gauss-Seidel         (Sec. 3)
  sgmg     multigrid on the full SG system, field-split smoother (Sec. 3)
  gmres    restarted (flexible) GMRES with right preconditioning (Sec. 3)
  mc       Monte Carlo / collocation reference statistics        (Sec. 2)
  cnn      mode-channel CNN forward/backward/Adam reference
  learned  the learned stage's composition with the field split

Parity status of each function is stated in its module docstring; every
function here is pinned by a `-m "not gpu"` test against closed forms,
quadrature brute force, invariants or a direct solve.
"""
