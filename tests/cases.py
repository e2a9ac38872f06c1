"""Test helpers: the seeded workloads (re-exported from the package), sampled
output indices, the oracle at sampled outputs and the parity measures."""
from __future__ import annotations

from oracle.compare import check, errors, max_err, rel_err  # noqa: F401
from oracle.sampled import sampled_adjoint, sampled_response  # noqa: F401
from paper_2204_06633_amd.inputs import sample_indices  # noqa: F401
from paper_2204_06633_amd.workloads import Case, day_case, make_case, year_case  # noqa: F401


def oracle_sampled_response(orb_p, orb_t, case, out_idx):
    return sampled_response(orb_p, orb_t, case, out_idx)
