"""Proposition 1 on the device as a function of the batch size (a
measurement, not a test: `python -m tests.measure_variance` on a GPU prints
one JSON line).  Lives under tests/ because it runs the oracle's closed forms."""
import json
import sys


def note(msg):
    print("[variance] " + msg, file=sys.stderr, flush=True)


def variance_study(torch, B=4000):
    """Proposition 1 on the device: 200 random neutral charges in a 10^3 box
    (reduced units, alpha = 0.3), the FP64 device estimator over B batches for
    p = 4 .. 256: empirical variance of F* (summed over particles) and of the
    isotropic P2*, against the closed forms eq. (ForceExp) / (PressExp) the
    oracle evaluates from the full Ewald sum."""
    from tests.test_gpu_variance import system, closed_forms, gpu_moments
    dev = torch.device("cuda:0")
    s = system()
    out = []
    for p in (4, 16, 64, 256):
        var_f, F1, var_p, P2 = closed_forms(s, p)
        sf, sf2, sp, sp2 = gpu_moments(s, p, B, dev, system_id=7000 + p)
        empF = (sf2 / B - (sf / B) ** 2).sum()
        empP = sp2 / B - (sp / B) ** 2
        out.append({"p": p, "batches": B, "force_var_closed": float(var_f.sum()),
                    "force_var_device": float(empF), "pressure_var_closed": float(var_p),
                    "pressure_var_device": float(empP)})
        note("variance p=%d: force %.4g / %.4g, pressure %.4g / %.4g"
             % (p, empF, var_f.sum(), empP, var_p))
    return out


if __name__ == "__main__":
    import torch
    print(json.dumps({"variance_study": variance_study(torch)}), flush=True)
