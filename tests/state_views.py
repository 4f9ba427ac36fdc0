"""Views of a run's stored state without the padding between planes.

lbm_cde_get_state copies whole population planes, including the padding the
library leaves between them (never written, so its bytes are whatever the
workspace held); comparisons of states must look at the nodes only."""
import numpy as np

ELEM = {"fp64": 8, "fp32": 4, "fp16": 2, "fp16_literal": 2}


def populations(state: np.ndarray, Q: int, nodes: int, precision: str):
    """(Q, nodes) stored populations and, for FP16 split storage, phi (nodes)."""
    st = np.asarray(state)
    if precision == "fp16":
        plane = (st.size - 4 * nodes) // (Q * 2)
        pops = st[:Q * plane * 2].view(np.float16).reshape(Q, plane)[:, :nodes]
        phi = st[Q * plane * 2:Q * plane * 2 + 4 * nodes].view(np.float32)
        return pops.copy(), phi.copy()
    dt = {8: np.float64, 4: np.float32, 2: np.float16}[ELEM[precision]]
    plane = st.size // (Q * ELEM[precision])
    return st.view(dt).reshape(Q, plane)[:, :nodes].copy(), None
