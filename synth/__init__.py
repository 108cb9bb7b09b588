"""Seeded synthetic inputs (symbols, received WDM fields) for tests and benchmarks."""
from .field import (WdmSpec, ChannelSpec, received_field, random_field, qam_symbols,  # noqa: F401
                    rrc_amplitude, rng_for, wdm_transmit, manakov_link)
from .workloads import WORKLOADS, workload  # noqa: F401
