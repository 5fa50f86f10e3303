"""Shared helpers of the test suite (no method arithmetic)."""
import numpy as np


def rel_err(a, b):
    """Normwise relative error max|a - b| / max|b| (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if a.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    return torch.device("cuda:0")


def dev_case(case, precision="f64", u0=None):
    """Device tensors of a case's inputs for the HIP path."""
    import torch
    d = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    f64 = torch.float64
    src = case.u0 if u0 is None else u0
    u = None if src is None else torch.as_tensor(src, dtype=f64).to(d).to(T).contiguous()
    out = dict(
        u=u,
        f=None if u is None else torch.zeros_like(u),
        xp=torch.as_tensor(case.xp, dtype=f64).to(d).contiguous(),
        up=torch.as_tensor(case.up, dtype=f64).to(d).contiguous(),
        wp=torch.as_tensor(case.wp, dtype=f64).to(d).contiguous(),
        radius=torch.as_tensor(case.radius, dtype=f64).to(d).contiguous(),
        mass=torch.as_tensor(case.mass, dtype=f64).to(d).contiguous(),
        body=torch.as_tensor(case.body, dtype=f64).to(d).contiguous(),
        dV=torch.as_tensor(case.dV, dtype=f64).to(d).contiguous(),
    )
    return out


def gpu_forcing(case, precision="f64", mask=None, want_U=False, params=None, u0=None, plan=None):
    """Run ibmx_forcing once on a case; returns numpy results."""
    import torch
    from paper_2109_03972_amd import ibmx
    prm = dict(case.params if params is None else params)
    D = dev_case(case, precision, u0=u0)
    if plan is None:
        plan = ibmx.Plan.from_case(case, precision, params=prm)
        plan.set_markers(D["body"], D["dV"])
    n_iter = int(prm["n_iter"])
    resid = torch.zeros(n_iter + 1, dtype=torch.float64, device=D["u"].device)
    U = None
    if want_U:
        U = torch.zeros((n_iter, 3, case.nm), dtype=D["u"].dtype, device=D["u"].device)
    mk = None
    if mask is not None:
        mk = torch.as_tensor(np.ascontiguousarray(mask, dtype=np.uint8)).to(D["u"].device)
    S, T = plan.forcing(D["u"], D["f"], D["xp"], D["up"], D["wp"], mask=mk, resid=resid, U_debug=U)
    st = plan.status()
    torch.cuda.synchronize()
    res = dict(u=D["u"].double().cpu().numpy(), f_tot=D["f"].double().cpu().numpy(),
               S=S.cpu().numpy(), T=T.cpu().numpy(), resid=resid.cpu().numpy(), status=st,
               stats=plan.stats())
    if want_U:
        res["U"] = U.double().cpu().numpy()
    return res
