"""Seeded synthetic inputs (symbols, received WDM fields) for tests and benchmarks."""
from .field import (WdmSpec, ChannelSpec, received_field, random_field, qam_symbols,  # noqa: F401
                    rrc_amplitude, rng_for, wdm_transmit, manakov_link, select_channel)
from .workloads import WORKLOADS, dbp_rate, workload  # noqa: F401
