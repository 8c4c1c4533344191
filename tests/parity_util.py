"""Helpers shared by the GPU parity tests: oracle <-> C-ABI state conversion
and the error norms the tolerances are stated in."""
import numpy as np

from oracle import qsp_oracle as O

FIELD_NAMES = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz")
DEPOSIT_NAMES = ("rho_mjz", "jx", "jy", "jz", "rho")


def oracle_state_to_abi(cfg, st):
    """The oracle's SliceState in the C-ABI layout (w per cell area)."""
    p = st.plasma
    return {"x": p.x, "y": p.y, "ux": p.ux, "uy": p.uy, "psi": p.psi,
            "w": p.w / (cfg.hx * cfg.hy), "hist": p.hist,
            "jx_prev": st.jx_prev, "jy_prev": st.jy_prev,
            "bx_prev1": st.bx_prev1, "by_prev1": st.by_prev1,
            "bx_prev2": st.bx_prev2, "by_prev2": st.by_prev2}


def rel_l2(a, ref, scale=None):
    """||a - ref|| / ||ref|| over interior nodes (or / scale)."""
    d = np.asarray(a, dtype=np.float64)[..., 1:-1, 1:-1] - np.asarray(ref)[..., 1:-1, 1:-1]
    den = np.linalg.norm(np.asarray(ref)[..., 1:-1, 1:-1]) if scale is None else scale
    return float(np.linalg.norm(d) / den) if den > 0 else float(np.linalg.norm(d))


def field_errors(gpu: dict, ref: dict):
    """Per-quantity rel-L2; Bz (O(h^2) for round beams) is measured against
    the norm of (Bx, By)."""
    out = {}
    bperp = np.sqrt(np.linalg.norm(np.asarray(ref["bx"])[..., 1:-1, 1:-1]) ** 2 +
                    np.linalg.norm(np.asarray(ref["by"])[..., 1:-1, 1:-1]) ** 2)
    for q in gpu:
        out[q] = rel_l2(gpu[q], ref[q], bperp if q == "bz" else None)
    return out
