"""Differentiable hull volume and surface area (torch.autograd.Function).

Forward and backward both run in the HIP library (hull_volume_area_fwd /
hull_volume_area_bwd); this module only connects them to autograd.  The face
set is fixed input data (for instance from hull_full on the int32-snapped
points) and carries no gradient.
"""
import torch

from . import hull


def _c(t, dtype):
    return t if (t.dtype == dtype and t.is_contiguous()) else t.to(dtype).contiguous()


class HullVolArea(torch.autograd.Function):
    """V, A = HullVolArea.apply(p, pt_off, faces, face_off)

    p        float32 [N, 3] CUDA (clouds concatenated)
    pt_off   int64 [H + 1] CUDA, point offsets of the clouds
    faces    int32 [F, 3] CUDA, outward faces with cloud-local indices
    face_off int64 [H + 1] CUDA, face offsets of the clouds
    returns  V, A: float32 [H]
    """

    @staticmethod
    def forward(ctx, p, pt_off, faces, face_off):
        p = _c(p, torch.float32)
        pt_off = _c(pt_off, torch.int64)
        faces = _c(faces, torch.int32)
        face_off = _c(face_off, torch.int64)
        V, A = hull.volume_area_fwd(p, pt_off, faces, face_off)
        ctx.save_for_backward(p, pt_off, faces, face_off)
        ctx.mark_non_differentiable()
        return V, A

    @staticmethod
    def backward(ctx, gV, gA):
        p, pt_off, faces, face_off = ctx.saved_tensors
        gV = _c(gV, torch.float32) if gV is not None else None
        gA = _c(gA, torch.float32) if gA is not None else None
        g = hull.volume_area_bwd(p, pt_off, faces, face_off, gV, gA)
        return g, None, None, None


def volume_area(p, pt_off, faces, face_off):
    return HullVolArea.apply(p, pt_off, faces, face_off)
