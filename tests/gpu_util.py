"""Helpers for GPU tests: scene upload and oracle comparison (inputs only)."""
import numpy as np
import torch

import paper_2404_09531_amd as om

DEV = "cuda:0"


def upload_scene(sc, dtype=torch.float32, device=DEV):
    """Device copies of a scenegen-style scene dict; returns (Scene, tensors)."""
    t = {}
    for k in ("grid", "plane_xy", "plane_xz", "plane_yz"):
        x = torch.from_numpy(np.ascontiguousarray(sc[k], dtype=np.float32)).to(device)
        t[k] = om.to_bf16(x) if dtype == torch.bfloat16 else x
    t["occ"] = torch.from_numpy(np.ascontiguousarray(sc["occ"], dtype=np.float32)).to(device)
    t["mlp"] = torch.from_numpy(np.ascontiguousarray(sc["mlp"], dtype=np.float32)).to(device)
    scene = om.Scene(t["grid"], t["plane_xy"], t["plane_xz"], t["plane_yz"], t["occ"], t["mlp"],
                     box_lo=tuple(float(v) for v in sc["box_lo"]), box_hi=tuple(float(v) for v in sc["box_hi"]))
    return scene, t


def rays_to(o, d, device=DEV):
    return (torch.from_numpy(np.ascontiguousarray(o, np.float32)).to(device),
            torch.from_numpy(np.ascontiguousarray(d, np.float32)).to(device))


def bf16_round(a):
    """float32 -> bfloat16 -> float32 (round to nearest even), on the CPU."""
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).float().numpy()


def log(msg):
    print(msg, flush=True)
