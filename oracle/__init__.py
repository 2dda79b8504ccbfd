"""CPU oracle for the Robust-l0 decoder (Mendoza-Smith, Tanner, Wechsung, arXiv 1704.09012).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the CPU
baseline leg of the benchmark may import anything from this package.  The product
path (the HIP library and its Python binding) never calls it, and it never calls the
product path: the two share no code.  The only common module is the seeded instance
generator, which holds no arithmetic of the method.

Modules
  posterior  -- the asymptotic posteriors p_z, p_e for Gaussian signal and noise
                (Thm. "Probabilities ...", eq:pz_gaussian / eq:pe_gaussian), their
                truncated-series-plus-Gaussian-tail approximations (eq:pz_approx /
                eq:pe_approx) and the normalised forms of eq:breve.  fp64.
  scores     -- the score tables the decoder evaluates, the t-sweep schedule, the
                rule for c (eq:finetune_c_cont / eq:finetune_c_quant) and the
                stopping tolerance (Sec. 4 "Stopping conditions").
  decoder    -- Robust-l0 (Alg. 1) and its noiseless reduction Parallel-l0 (Alg. 2),
                step by step, in the float32 contract stated in its header.
  bruteforce -- exhaustive l0 minimisation for tiny n (the problem statement of Sec. 1).
  mlp        -- the learned accept/value network (not from the paper), fp64 forward,
                manual backward and a bf16-emulating inference.
"""
