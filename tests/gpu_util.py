"""Helpers shared by the GPU tests: move seeded inputs to the device and run
the engine through the C ABI binding."""
import numpy as np

from paper_1809_08857_amd import mg


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_solver(p, **desc_kw):
    eps = dev(p.eps) if p.eps is not None else None
    faces = tuple(dev(a) for a in p.faces) if getattr(p, "faces", None) is not None else None
    return mg.Solver(p.nx, p.ny, p.nz, p.h, eps=eps, faces=faces, a=p.a, bc_types=p.bc_types(),
                     bc_values=p.bc_values(), **desc_kw)


def gpu_solve(p, x0=None, flags=0, **desc_kw):
    """(x as numpy, rc, stats dict)."""
    import torch
    s = make_solver(p, **desc_kw)
    try:
        f = dev(p.f)
        x = dev(x0) if x0 is not None else torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        rc, st = s.solve(f, x, flags)
        torch.cuda.synchronize()
        return x.cpu().numpy(), rc, st.as_dict()
    finally:
        s.close()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
