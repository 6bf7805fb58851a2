#!/usr/bin/env python
"""Studies around the minSR hot path on one MI355X, each printing JSON lines.

  stability   The training-instability grid of App. E (Fig. 6): the 1D
              transverse-field Ising chain (N = 200, open, J = h = 1) with a
              1D GRU pRNN of d_h = 32, trained for 100 minSR steps from the
              seeded initialisation for every shift lambda and sample count
              Ns of a grid, in the FP64, BF16 + FP64 and plain FP32 forms
              (mu = 0.7 as the paper's 1D TFIM runs; eta = 0.05: at the
              paper's 0.5 most runs of this initialisation collapse into the
              ferromagnetic product state within a few steps, where T = 0,
              which says nothing about the solve).  Per run:
              the steps that failed (non-finite local energies or update,
              a non-positive Cholesky pivot: the step is skipped), the first
              of them, the energy per site above the exact ground energy
              over the last 10 steps, and at the last step the condition
              number kappa_2(T + lambda I) with the digit estimate
              d = -log10(kappa_2 eps) for the form's machine epsilon.
  qgt         The subsampled-QGT error of Prop. 3 (Sec. 5, Fig. 5b) on the
              6 x 6 open J1-J2 model (J2 = 0.5) with a 2D cRNN at
              initialisation: the parameter-space metric S~ = O' O'^T of Ns
              samples against a reference S from Ns_ref samples, as
              ||S - S~||_F / ||S||_F against alpha = sqrt(Ns) / N_p, with the
              bound alpha^-1 sqrt(V_avg / epsilon) of Eq. UB, V_avg estimated
              from the reference samples.

Inputs are synthetic: the method draws its own samples.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# exact ground energy per site of the open critical chain with N = 200
# (the paper's reference value for its 1D TFIM benchmark, Table 2)
E0_TFIM200_PER_SITE = -1.27142590795


def stability(args):
    import numpy as np
    import torch
    import paper_2608_18065_amd as pm
    N, H = 200, 32
    lams = [float(x) for x in args.lams.split(",")]
    nss = [int(x) for x in args.ns.split(",")]
    forms = [("fp64", pm.FORM_FP64_REF, "f64", 2.0 ** -52),
             ("bf16_fp64", pm.FORM_BF16_FP64, "f32", 2.0 ** -24),
             ("fp32_plain", pm.FORM_FP32_PLAIN, "f32", 2.0 ** -23)]
    if args.forms:
        keep = args.forms.split(",")
        forms = [f for f in forms if f[0] in keep]
    ham = pm.hamiltonian("tfim", J=1.0, h=1.0, pbc=False)
    K = args.steps
    for fname, form, dtype, eps in forms:
        for Ns in nss:
            for lam in lams:
                m = pm.Model(N, 1, 1, H, dtype=dtype, seed=2100, max_Ns=Ns, pinv=True)
                mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
                outs = m.step_outputs(Ns)
                hist = torch.zeros((K, 3), dtype=torch.float64, device="cuda")
                st = torch.zeros(K, dtype=torch.int32, device="cuda")
                t0 = time.perf_counter()
                for i in range(K):
                    m.step(ham, Ns, args.eta, lam, 0.7, mom, 1100, i, form=form, outputs=outs)
                    hist[i].copy_(outs["energy"], non_blocking=True)
                    st[i:i + 1].copy_(outs["status"], non_blocking=True)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                T = m.intermediates(form)["T"].double()
                w, cond, cst = m.spectrum(T, lam=lam, eps=eps)
                torch.cuda.synchronize()
                s = st.cpu().numpy()
                E = hist.cpu().numpy()[:, 0] / N
                bad = np.nonzero(s & pm.ST_ERRORS)[0]
                tailE = E[-10:]
                c = cond.cpu().numpy()
                print(json.dumps({
                    "study": "stability", "form": fname, "Ns": Ns, "lambda": lam, "steps": K,
                    "eta": args.eta,
                    "failed_steps": int(len(bad)),
                    "first_failed_step": int(bad[0]) if len(bad) else None,
                    "nonfinite_energy": bool(not np.all(np.isfinite(E))),
                    "dE_per_site_last10": float(np.mean(tailE) - E0_TFIM200_PER_SITE)
                    if np.all(np.isfinite(tailE)) else None,
                    "kappa2_last": float(c[2]), "digits_last": float(c[3]),
                    "eps": eps, "eig_status": int(cst.item()), "ms_per_step": sec / K * 1e3}),
                    flush=True)
                m.close()


def qgt(args):
    import numpy as np
    import torch
    import paper_2608_18065_amd as pm
    L, H = 6, 8
    ns_ref = args.ns_ref
    nss = [int(x) for x in args.ns.split(",")]
    m = pm.Model(L, L, 2, H, complex_head=True, marshall=True, dtype="f64", seed=2200,
                 max_Ns=max(ns_ref, max(nss)))
    Np = m.Np
    sig, _ = m.sample(ns_ref, key=1200, counter=0)
    S_ref = m.param_gram(sig)
    # V_avg = mean over (i, j) of Var(X_i X_j^*) from the reference samples,
    # X the population-centred log-derivatives (here: centred on the
    # reference mean); Var(Z) = E|Z|^2 - |E Z|^2
    O, _ = m.jacobian(sig)                        # rows: Re then Im, / sqrt(Ns_ref)
    O = O * math.sqrt(ns_ref)
    X = torch.complex(O[:ns_ref], O[ns_ref:])
    X = X - X.mean(dim=0, keepdim=True)
    Q = (X.T @ X.conj()) / ns_ref
    A = (X.abs() ** 2).to(torch.float64)
    M = (A.T @ A) / ns_ref
    v_avg = float((M - Q.abs() ** 2).mean().item())
    s_norm = float(torch.linalg.norm(S_ref).item())
    for Ns in nss:
        errs = []
        for rep in range(args.reps):
            sg, _ = m.sample(Ns, key=1300 + rep, counter=Ns)
            S = m.param_gram(sg)
            errs.append(float(torch.linalg.norm(S - S_ref).item()) / s_norm)
        alpha = math.sqrt(Ns) / Np
        bound = math.sqrt(v_avg / args.epsilon) / alpha / s_norm
        print(json.dumps({"study": "qgt", "L": L, "d_h": H, "Np": Np, "Ns": Ns,
                          "Ns_ref": ns_ref, "alpha": alpha,
                          "rel_err_mean": float(np.mean(errs)), "rel_err_max": float(np.max(errs)),
                          "reps": args.reps, "bound_rel": bound, "epsilon": args.epsilon,
                          "V_avg": v_avg}), flush=True)
    m.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="study", required=True)
    a = sub.add_parser("stability")
    a.add_argument("--lams", default="1e-6,1e-5,1e-4,1e-3,1e-2,1e-1")
    a.add_argument("--ns", default="50,100,200,400,800")
    a.add_argument("--forms", default="")
    a.add_argument("--steps", type=int, default=100)
    a.add_argument("--eta", type=float, default=0.05)
    b = sub.add_parser("qgt")
    b.add_argument("--ns", default="16,32,64,128,256,512,1024")
    b.add_argument("--ns-ref", type=int, default=8192)
    b.add_argument("--reps", type=int, default=4)
    b.add_argument("--epsilon", type=float, default=1e-6)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    {"stability": stability, "qgt": qgt}[args.study](args)


if __name__ == "__main__":
    main()
