"""Host checks of the synthetic input generator: crops and frame subsets
reproduce the full clip bit for bit, and the disc-outline distance used to
split events at moving edges from the rest marks exactly the pixels whose
samples straddle two surfaces."""
import numpy as np
import torch

from paper_2303_02608_amd import synth


def _spec():
    return synth.config_spec(0)["spec"]


def test_crops_and_frame_subsets_reproduce_the_full_clip():
    s = _spec()
    full = synth.make_clip(s)
    part = synth.make_clip(s, frames=[3, 7, 8], crop=(5, 9, 20, 17))
    for k in ("E", "var"):
        assert torch.equal(part[k], full[k][[3, 7, 8], 9:26, 5:25])
    assert torch.equal(part["feat"], full["feat"][[3, 7, 8], :, 9:26, 5:25])


def test_boundary_distance_against_sampled_outlines():
    s = _spec()
    scene = synth._Scene(s, torch.device("cpu"))
    T, H, W = s.T, s.H, s.W
    tt, yy, xx = torch.meshgrid(torch.arange(T), torch.arange(H), torch.arange(W), indexing="ij")
    d = synth.boundary_distance(s, tt, xx, yy).numpy()
    ang = np.linspace(0.0, 2 * np.pi, 4096, endpoint=False)
    tf = torch.arange(T, dtype=torch.float64)
    for t in (0, 9, 15):
        px, py = xx[t].numpy() + 0.5, yy[t].numpy() + 0.5
        best = np.full(px.shape, np.inf)
        for k, disc in enumerate(scene.discs):
            cx, cy = (v[t].item() for v in scene.disc_states(k, tf)[:2])
            ox, oy = cx + disc["R"] * np.cos(ang), cy + disc["R"] * np.sin(ang)
            dk = np.min(np.hypot(px[..., None] - ox, py[..., None] - oy), axis=-1)
            best = np.minimum(best, dk)
        # the nearest outline point is within an arc of R pi / 4096 of a
        # sampled one (triangle inequality)
        assert np.all(d[t] <= best + 1e-9)
        assert np.all(best - d[t] <= max(dd["R"] for dd in scene.discs) * np.pi / 4096 + 1e-9)


def test_boundary_distance_marks_mixed_pixels():
    """Sub-pixel samples lie within sqrt(2)/2 of the pixel centre, so a pixel
    farther than 0.75 px from every outline sees one surface only: its depth
    is the background's (>= 10) or a disc's (<= 6), never a mixture."""
    s = _spec()
    d = synth.make_clip(s)
    bound = 10.0 + 0.01 * s.H + 0.5 * s.bump_amp
    depth = d["feat"][:, 6].double().numpy() * bound
    T, H, W = depth.shape
    tt, yy, xx = torch.meshgrid(torch.arange(T), torch.arange(H), torch.arange(W), indexing="ij")
    dist = synth.boundary_distance(s, tt, xx, yy).numpy()
    mixed = (depth > 6.0 + 1e-4) & (depth < 10.0 - 1e-4)
    assert not np.any(mixed & (dist > 0.75))
    assert np.any(mixed)
