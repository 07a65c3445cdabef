"""Plain, slow FP64 CPU oracle for the local ETKF frame of Gray et al.,
"Local ensemble transform Kalman filter, a fast non-stationary control law for
adaptive optics on ELTs" (arXiv:1408.7069).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code, constants or helpers with the GPU path: the two meet only
through the seeded synthetic inputs.

Modules
  geometry    pupil mask, actuator grid, Fried slope operator, domains, taper
  letkf       forecast, per-domain analysis (three independent forms), gather
  kalman      brute-force Kalman update (the exact limit the ETKF must reach),
              the DARE gain and the stationary KF closed loop (the reference)
  philox      Philox4x32-10 counter-based generator and the noise-bank lookup
  accounting  the paper's operation counts (App. B, Tables 1, 3, 4)
  piston      least-squares differential-piston removal after the gather
  adjoint     hand-written reverse-mode gradient of the residual-variance loss
  delayed     the paper's state [phi_k; phi_{k-1}] with the measurement delay,
              the DM term of the observation and the command u_k
  metrics     coherent energy and the loss against the KF (Sec. 5)
  ar2         the AR(2) turbulence model from each member's last two analyses
  refit       online least-squares refit of the AR(1) coefficient and the
              model-noise scale that follows it (Sec. 4.2)
  blend       blend-mode gather: patch analyses put on a common piston and
              averaged with tent weights (a variant of the Sec. 4.2 gather)
  cl          covariance localisation (Sec. 4): the patch covariance tapered
              by a Schur product, Kalman gain in slope space, deterministic
              EnKF anomalies
"""
