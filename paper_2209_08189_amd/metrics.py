"""Registration quality measures of the paper's evaluation (Section 5.1,
measures of performance): Dice coefficients of label maps and the relative
mismatch.  Reporting helpers around the library; not part of the solver.

* D(l0, l1) = 2 |l0 & l1| / (|l0| + |l1|) per label;
* D_a: plain average over the foreground labels; D_vw: weighted by the
  label volumes |l1^i| of the reference; D_ivw: weighted by 1 / |l1^i|.
* Label warping: the indicator of every label is transported by the forward
  semi-Lagrangian solve with the velocity (tricubic), and each voxel takes
  the label of the largest transported indicator (ties to the lower label).
"""
import numpy as np


def dice(la, lb, labels=(1, 2, 3)):
    """Dice statistics of integer label maps la (warped template) and lb
    (reference), numpy or torch, over the given foreground labels."""
    la = _np(la)
    lb = _np(lb)
    D, vol = [], []
    for i in labels:
        a, b = la == i, lb == i
        na, nb = int(a.sum()), int(b.sum())
        D.append(2.0 * int(np.logical_and(a, b).sum()) / (na + nb) if na + nb else 1.0)
        vol.append(nb)
    D = np.array(D)
    vol = np.array(vol, dtype=np.float64)
    inv = np.where(vol > 0, 1.0 / np.maximum(vol, 1.0), 0.0)
    return {"D": D.tolist(), "D_a": float(D.mean()),
            "D_vw": float((vol * D).sum() / vol.sum()) if vol.sum() else 1.0,
            "D_ivw": float((inv * D).sum() / inv.sum()) if inv.sum() else 1.0}


def warp_labels(labels, v, nlabels=4, reg=None):
    """Label map transported by the velocity v (device tensor [3, n1, n2, n3])
    through the library's forward semi-Lagrangian solve; returns a device
    uint8 tensor.  reg: an existing context of the same grid to use (its
    images are replaced; v = None keeps its current velocity), else a
    temporary one."""
    import torch
    from .claire import Registration
    lab = torch.as_tensor(_np(labels)).cuda()
    shape = tuple(lab.shape)
    own = reg is None
    if own:
        reg = Registration(shape)
    if v is not None:
        reg.set_velocity(v)
    best = None
    arg = torch.zeros(shape, dtype=torch.uint8, device="cuda")
    for i in range(nlabels):
        ind = (lab == i).float()
        reg.set_images(ind, ind)
        del ind
        w = reg.deformed_template()
        # running argmax; ties keep the lower label
        if best is None:
            best = w
        else:
            take = w > best
            torch.maximum(best, w, out=best)
            arg[take] = i
            del take, w
    if own:
        reg.close()
    return arg


def relative_mismatch(m1, mt, m0):
    """r = ||m(1) - m1||^2 / ||m0 - m1||^2."""
    import torch
    return float(((mt - m1).double() ** 2).sum() / ((m0 - m1).double() ** 2).sum())


def _np(x):
    if hasattr(x, "detach"):
        import torch
        if x.is_cuda:
            torch.cuda.synchronize()
        return x.detach().cpu().numpy()
    return np.asarray(x)
