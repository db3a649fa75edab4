"""Node-by-node comparison used by the GPU parity tests."""
import numpy as np


def per_node_ok(got, ref, rel=1e-11, floor=1e-14):
    """Every node within rel of its own L2 norm, plus floor times the largest node's norm (nodes whose
    output cancels to a small value carry the rounding of their terms): a global norm alone could
    hide a wrong node of small norm.  Prints the worst ratio of error to own norm."""
    got = np.asarray(got).reshape(len(got), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    err = np.linalg.norm(got - ref, axis=1)
    nrm = np.linalg.norm(ref, axis=1)
    big = nrm.max()
    sized = nrm > 1e-6 * big
    worst = float(np.max(err[sized] / nrm[sized])) if sized.any() else 0.0
    print("per-node: worst error / own norm %.2e over the %d of %d nodes above 1e-6 of the largest; "
          "worst error / largest norm %.2e" % (worst, int(sized.sum()), ref.shape[0], float(err.max() / big)), flush=True)
    return bool(np.all(err <= rel * nrm + floor * big))
