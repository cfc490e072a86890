"""Device-resident MD-like loop: SASA and nonpolar forces every frame.

Coordinates, radii and outputs stay in HBM across frames.  Each frame moves
every atom by Gaussian noise (sigma A per component, drawn on the device from
a per-frame seeded generator), then the library computes per-atom SASA and the
nonpolar forces F = -gamma dA/dx (nonpolar energy gamma * SASA with one surface
tension for all atoms).  Nothing crosses to the host except the coordinates of
the frames the caller asks to keep.
"""
import time

import torch

from .context import SasaContext


def md_loop(xyz, radii, frames, sigma=0.02, gamma=0.005, seed=33, probe=1.4, precision="mixed",
            keep_frames=(), ctx=None, frame_hints=False):
    """Run ``frames`` frames; return per-frame latencies (ms) and the kept frames.

    keep_frames: frame indices whose coordinates, areas and forces are copied to
    the host (for checks against the oracle).
    frame_hints: use the library's trajectory mode (each atom's cell verified
    and kept from the previous frame, or clipped with its previous facets
    first; results equal up to the order of the sums).  Off by default: at
    0.02 A moves a frame keeps about half of the cells, which saves cuts but
    not the side tests of the remaining planes, and the mode's bookkeeping
    makes it no faster than clipping every cell from scratch.
    """
    dev = torch.device("cuda", torch.cuda.current_device())
    X = torch.as_tensor(xyz, dtype=torch.float64, device=dev).clone()
    R = torch.as_tensor(radii, dtype=torch.float64, device=dev).contiguous()
    ctx = ctx or SasaContext(device=dev.index, precision=precision, max_atoms=X.shape[0], frames=frame_hints)
    gen = torch.Generator(device=dev)
    kept = {}
    lat = []
    keep = set(keep_frames)
    noise = torch.empty_like(X)
    # the areas and forces of every frame land in the same two device buffers
    out = (torch.empty(X.shape[0], dtype=torch.float64, device=dev), torch.empty_like(X))
    for f in range(frames):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gen.manual_seed(seed * 1_000_003 + f)
        noise.normal_(0.0, sigma, generator=gen)
        X.add_(noise)
        area, forces = ctx.forces(X, R, gamma, probe, out=out)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t0))
        if f in keep:
            kept[f] = (X.cpu().numpy(), area.cpu().numpy(), forces.cpu().numpy())
    return lat, kept
