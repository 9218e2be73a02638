"""Seeded synthetic inputs shared by the GPU path and the oracle.

Holds workload shapes, replay-buffer generators and initial parameters only;
none of the method's arithmetic lives here.
"""
from .workloads import Workload, ALL as WORKLOADS  # noqa: F401
from .buffers import make_buffer, buffer_for  # noqa: F401
from .params import critic_params, critic_params_for, actor_params, mlp_layers  # noqa: F401
