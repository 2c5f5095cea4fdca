"""Error measures shared by the GPU parity tests (not a test module)."""
import numpy as np

STATE = ["step", "xc", "yc", "theta", "ux", "uy", "omega", "fx", "fy", "torque", "fx_hydro", "fy_hydro",
         "m_hydro", "fx_bond", "fy_bond", "m_bond", "fy_wall", "gap", "n_bonds", "n_probing"]


def col(name):
    return STATE.index(name)


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def trace_errors(tg, to, particle):
    """Relative errors of a particle series against the oracle's: vectors (velocity, force,
    displacement from the start) by their norm, the angle and angular velocity alone, the
    torque against |M| + a |F| (a the semi-major axis), so that components that are pure
    round-off do not pose as parity errors."""
    x0 = np.array([particle["xc"], particle["yc"]])
    U, X, F = [col("ux"), col("uy")], [col("xc"), col("yc")], [col("fx"), col("fy")]
    e = {"U": rel(tg[:, U], to[:, U]), "X": rel(tg[:, X] - x0, to[:, X] - x0),
         "theta": rel(tg[:, col("theta")], to[:, col("theta")]),
         "omega": rel(tg[:, col("omega")], to[:, col("omega")]), "F": rel(tg[:, F], to[:, F])}
    scale = np.linalg.norm(to[:, col("torque")]) + particle["a_major"] * np.linalg.norm(to[:, F])
    e["M"] = float(np.linalg.norm(tg[:, col("torque")] - to[:, col("torque")]) / scale) if scale > 0 else 0.0
    return e
